// Even-odd (checkerboard) form of D_W (the eo-decomposition the paper names as
// a next tuning step in Sec. 4).  With all extents even, parity(x) =
// (x + y + z + t) mod 2 splits the lattice into two checkerboards and every
// hop of D_W connects opposite parities:
//   D_W = [[A, H_eo], [H_oe, A]],  A = 4 + m0,
//   H psi(x) = -1/2 sum_mu [(1 - gamma_mu) V_mu(x) psi(x+mu) + (1 + gamma_mu) V_mu(x-mu)^dag psi(x-mu)].
// Packed layout of parity p: [Nt][Nz][Ny][Nx/2][...]; in row (y, z, t) the
// packed index i holds x = 2 i + r, r = (p + y + z + t) mod 2.  For an output
// site of parity p its x + 1 neighbour (parity 1 - p, same row) has packed
// index i + r and its x - 1 neighbour i - 1 + r (both mod Nx/2); the y, z, t
// neighbours keep the packed index i in the neighbour row.
#include "launch.hpp"
#include "stencils.hpp"

namespace dsl {

EoGeom make_eo_geom(const int dims[4], int nv) {
  EoGeom e;
  for (int i = 0; i < 4; ++i) e.n[i] = dims[i];
  e.nh = dims[0] / 2;
  e.hvol = uint32_t(e.nh) * dims[1] * dims[2] * dims[3];
  e.nv = nv;
  e.dnh = FastDiv::make(e.nh);
  e.dy = FastDiv::make(dims[1]);
  e.dz = FastDiv::make(dims[2]);
  return e;
}

// ---------------------------------------------------------------- packing
// Copies the `words` storage words of every site of parity p between the full
// and the packed layout, in 16-byte pieces (words * word bytes is a multiple of
// 16 for every field of the library: 12 N_v or 3 N_v complex spinors with
// N_v even, and the 36-word link blocks; odd block sizes use 8 or 4 bytes).
template <class P, bool TO_PACKED>
__global__ void __launch_bounds__(256) eo_copy_kernel(EoGeom e, int p, const P* __restrict__ src, P* __restrict__ dst,
                                                      int pieces) {
  const size_t total = size_t(e.hvol) * pieces;
  for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < total; k += size_t(gridDim.x) * blockDim.x) {
    const uint32_t q = uint32_t(k / pieces);
    const int j = int(k - size_t(q) * pieces);
    const uint32_t row = e.dnh.div(q);
    const uint32_t i = q - row * uint32_t(e.nh);
    const uint32_t yzt = row;
    const uint32_t zt = e.dy.div(yzt);
    const uint32_t y = yzt - zt * uint32_t(e.n[1]);
    const uint32_t t = e.dz.div(zt);
    const uint32_t z = zt - t * uint32_t(e.n[2]);
    const uint32_t r = (uint32_t(p) + y + z + t) & 1u;
    const size_t full = size_t(row) * e.n[0] + 2 * i + r;
    if (TO_PACKED)
      dst[size_t(q) * pieces + j] = src[full * pieces + j];
    else
      dst[full * pieces + j] = src[size_t(q) * pieces + j];
  }
}

hipError_t launch_eo_copy(bool to_packed, const EoGeom& e, int parity, const void* src, void* dst, size_t site_bytes,
                          hipStream_t st) {
  size_t total;
  const dim3 block(256);
  auto grid_for = [&](size_t n) {
    size_t b = (n + 255) / 256;
    if (b > 65536) b = 65536;
    return dim3(unsigned(b > 0 ? b : 1));
  };
  if (site_bytes % 16 == 0) {
    const int pieces = int(site_bytes / 16);
    total = size_t(e.hvol) * pieces;
    if (to_packed)
      hipLaunchKernelGGL((eo_copy_kernel<u32x4, true>), grid_for(total), block, 0, st, e, parity, (const u32x4*)src,
                         (u32x4*)dst, pieces);
    else
      hipLaunchKernelGGL((eo_copy_kernel<u32x4, false>), grid_for(total), block, 0, st, e, parity, (const u32x4*)src,
                         (u32x4*)dst, pieces);
  } else if (site_bytes % 8 == 0) {
    const int pieces = int(site_bytes / 8);
    total = size_t(e.hvol) * pieces;
    if (to_packed)
      hipLaunchKernelGGL((eo_copy_kernel<u32x2, true>), grid_for(total), block, 0, st, e, parity, (const u32x2*)src,
                         (u32x2*)dst, pieces);
    else
      hipLaunchKernelGGL((eo_copy_kernel<u32x2, false>), grid_for(total), block, 0, st, e, parity, (const u32x2*)src,
                         (u32x2*)dst, pieces);
  } else {
    const int pieces = int(site_bytes / 4);
    total = size_t(e.hvol) * pieces;
    if (to_packed)
      hipLaunchKernelGGL((eo_copy_kernel<unsigned, true>), grid_for(total), block, 0, st, e, parity,
                         (const unsigned*)src, (unsigned*)dst, pieces);
    else
      hipLaunchKernelGGL((eo_copy_kernel<unsigned, false>), grid_for(total), block, 0, st, e, parity,
                         (const unsigned*)src, (unsigned*)dst, pieces);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- hop
// Empty register constraint on the accumulator after each hop: keeps the
// hops in sequence (the scheduler otherwise hoists every hop's operands and
// spills).
template <class T>
__device__ __forceinline__ void eo_hold(cpx<T> (&acc)[4][3]) {
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) asm volatile("" : "+v"(acc[a][c].r), "+v"(acc[a][c].i));
}

// out = c_add add + c_hop H in  on the packed sites of parity p (add may be
// null: then out = c_hop H in).  Uo: packed links of the parity-p sites
// (V_mu(x) of the forward hops); Ui: packed links of the parity 1 - p sites
// (V_mu(x - mu) of the backward hops).  One thread per (packed site, rhs).
template <bool ADJ, class S, class T>
__global__ void __launch_bounds__(256, 3) wilson_eo_hop_kernel(EoGeom e, int p, const typename S::word* __restrict__ Uo,
                                                            const typename S::word* __restrict__ Ui,
                                                            const typename S::word* __restrict__ in,
                                                            typename S::word* __restrict__ out,
                                                            const typename S::word* __restrict__ add, T c_add,
                                                            T c_hop) {
  constexpr int CF = ADJ ? +1 : -1;  // forward projector 1 + CF gamma
  constexpr int CB = -CF;            // backward projector 1 + CB gamma
  const uint32_t q = blockIdx.x * blockDim.y + threadIdx.y;
  const int v = blockIdx.y * blockDim.x + threadIdx.x;
  if (q >= e.hvol || v >= e.nv) return;
  const int nv = e.nv, nh = e.nh;
  const size_t sps = size_t(12) * nv;
  const uint32_t row = e.dnh.div(q);
  const int i = int(q - row * uint32_t(nh));
  const uint32_t zt = e.dy.div(row);
  const int y = int(row - zt * uint32_t(e.n[1]));
  const uint32_t tt = e.dz.div(zt);
  const int z = int(zt - tt * uint32_t(e.n[2]));
  const int t = int(tt);
  const int r = (p + y + z + t) & 1;
  int ixp = i + r, ixm = i - 1 + r;
  if (ixp >= nh) ixp -= nh;
  if (ixm < 0) ixm += nh;
  const int ny = e.n[1], nz = e.n[2], ntt = e.n[3];
  auto prow = [&](int yy, int zz, int tq) -> uint32_t { return uint32_t(yy + ny * (zz + nz * tq)) * uint32_t(nh); };
  const int yp = y + 1 == ny ? 0 : y + 1, ym = y == 0 ? ny - 1 : y - 1;
  const int zp = z + 1 == nz ? 0 : z + 1, zm = z == 0 ? nz - 1 : z - 1;
  const int tp = t + 1 == ntt ? 0 : t + 1, tm = t == 0 ? ntt - 1 : t - 1;
  const uint32_t qxp = row * uint32_t(nh) + ixp, qxm = row * uint32_t(nh) + ixm;
  const uint32_t qyp = prow(yp, z, t) + i, qym = prow(ym, z, t) + i;
  const uint32_t qzp = prow(y, zp, t) + i, qzm = prow(y, zm, t) + i;
  const uint32_t qtp = prow(y, z, tp) + i, qtm = prow(y, z, tm) + i;

  cpx<T> acc[4][3];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[a][c] = zero<T>();
  wilson_hop<0, CF, false, S, T>(Uo, in, (size_t(q) * 4 + 0) * 9, size_t(qxp) * sps + v, nv, acc);
  eo_hold<T>(acc);
  wilson_hop<0, CB, true, S, T>(Ui, in, (size_t(qxm) * 4 + 0) * 9, size_t(qxm) * sps + v, nv, acc);
  eo_hold<T>(acc);
  wilson_hop<1, CF, false, S, T>(Uo, in, (size_t(q) * 4 + 1) * 9, size_t(qyp) * sps + v, nv, acc);
  eo_hold<T>(acc);
  wilson_hop<1, CB, true, S, T>(Ui, in, (size_t(qym) * 4 + 1) * 9, size_t(qym) * sps + v, nv, acc);
  eo_hold<T>(acc);
  wilson_hop<2, CF, false, S, T>(Uo, in, (size_t(q) * 4 + 2) * 9, size_t(qzp) * sps + v, nv, acc);
  eo_hold<T>(acc);
  wilson_hop<2, CB, true, S, T>(Ui, in, (size_t(qzm) * 4 + 2) * 9, size_t(qzm) * sps + v, nv, acc);
  eo_hold<T>(acc);
  wilson_hop<3, CF, false, S, T>(Uo, in, (size_t(q) * 4 + 3) * 9, size_t(qtp) * sps + v, nv, acc);
  eo_hold<T>(acc);
  wilson_hop<3, CB, true, S, T>(Ui, in, (size_t(qtm) * 4 + 3) * 9, size_t(qtm) * sps + v, nv, acc);
  eo_hold<T>(acc);

  const T ch = T(-0.5) * c_hop;
  const size_t base = size_t(q) * sps + v;
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const size_t k = base + size_t(sp * 3 + c) * nv;
      cpx<T> o;
      o.r = ch * acc[sp][c].r;
      o.i = ch * acc[sp][c].i;
      if (add) {
        const cpx<T> a = S::template load<T>(add + k);
        o.r = fma(c_add, a.r, o.r);
        o.i = fma(c_add, a.i, o.i);
      }
      S::template store<T>(out + k, o);
    }
}

hipError_t launch_wilson_eo_hop(bool adj, int dtype, const EoGeom& e, int parity, const void* Uo, const void* Ui,
                                const void* in, void* out, const void* add, double c_add, double c_hop,
                                hipStream_t st, int epi, EpiArgs* ea) {
  const hipError_t rows =
      launch_wilson_eo_rows(adj, dtype, e, parity, Uo, Ui, in, out, add, c_add, c_hop, st, epi, ea);
  if (rows != hipErrorNotSupported || epi != EPI_STORE || knobs().rows.get(1) == 2) return rows;
  Shape sh = site_v_shape(e.hvol, e.nv);
#define DSL_EO(SS, TT)                                                                                          \
  do {                                                                                                           \
    using W = typename SS::word;                                                                                 \
    if (adj)                                                                                                     \
      hipLaunchKernelGGL((wilson_eo_hop_kernel<true, SS, TT>), sh.grid, sh.block, 0, st, e, parity,              \
                         (const W*)Uo, (const W*)Ui, (const W*)in, (W*)out, (const W*)add, TT(c_add), TT(c_hop)); \
    else                                                                                                         \
      hipLaunchKernelGGL((wilson_eo_hop_kernel<false, SS, TT>), sh.grid, sh.block, 0, st, e, parity,             \
                         (const W*)Uo, (const W*)Ui, (const W*)in, (W*)out, (const W*)add, TT(c_add), TT(c_hop)); \
  } while (0)
  switch (dtype) {
    case DT_C64: DSL_EO(C64, float); break;
    case DT_C128: DSL_EO(C128, double); break;
    case DT_BF16: DSL_EO(BF16, float); break;
    case DT_F16: DSL_EO(F16, float); break;
    default: return hipErrorInvalidValue;
  }
#undef DSL_EO
  return hipGetLastError();
}

}  // namespace dsl
