// Common device/host helpers of the Dirac-operator kernels (gfx950).
//
// * cpx<T>: complex arithmetic in the compute type T (float or double).
// * Storage tags C64, C128, BF16, F16: how one complex number sits in memory
//   and how it converts to and from the compute type (round to nearest even
//   on narrowing stores).
// * FastDiv: division by a run-time constant with one mul-hi, so that site
//   coordinates cost a handful of integer ops per thread.
// * Geom: lattice extents, site strides and the per-thread neighbour offsets
//   for periodic boundaries (site s = x + Nx (y + Ny (z + Nz t))).
// * xcd_block: reorders workgroups so that each of the 8 XCDs (each with its
//   own L2) walks a contiguous range of sites, which keeps the spinors of
//   neighbouring sites in that XCD's L2.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define DSL_HD __host__ __device__ __forceinline__

namespace dsl {

// 16 and 8 bytes as native vectors (HIP's uint4 is a class around a union,
// which keeps arrays of it in scratch memory instead of registers).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <class T>
struct cpx {
  T r, i;
};

template <class T> DSL_HD cpx<T> mk(T r, T i) { return cpx<T>{r, i}; }
template <class T> DSL_HD cpx<T> zero() { return cpx<T>{T(0), T(0)}; }
template <class T> DSL_HD cpx<T> operator+(cpx<T> a, cpx<T> b) { return {a.r + b.r, a.i + b.i}; }
template <class T> DSL_HD cpx<T> operator-(cpx<T> a, cpx<T> b) { return {a.r - b.r, a.i - b.i}; }
template <class T> DSL_HD cpx<T> operator-(cpx<T> a) { return {-a.r, -a.i}; }
template <class T> DSL_HD cpx<T> operator*(T s, cpx<T> a) { return {s * a.r, s * a.i}; }
template <class T> DSL_HD cpx<T>& operator+=(cpx<T>& a, cpx<T> b) { a.r += b.r; a.i += b.i; return a; }
template <class T> DSL_HD cpx<T>& operator-=(cpx<T>& a, cpx<T> b) { a.r -= b.r; a.i -= b.i; return a; }
// i * a and -i * a
template <class T> DSL_HD cpx<T> times_i(cpx<T> a) { return {-a.i, a.r}; }
template <class T> DSL_HD cpx<T> times_mi(cpx<T> a) { return {a.i, -a.r}; }
template <class T> DSL_HD cpx<T> conj(cpx<T> a) { return {a.r, -a.i}; }
// acc + a * b
template <class T> DSL_HD cpx<T> cmadd(cpx<T> acc, cpx<T> a, cpx<T> b) {
  acc.r = fma(a.r, b.r, acc.r);
  acc.r = fma(-a.i, b.i, acc.r);
  acc.i = fma(a.r, b.i, acc.i);
  acc.i = fma(a.i, b.r, acc.i);
  return acc;
}
// acc + conj(a) * b
template <class T> DSL_HD cpx<T> cjmadd(cpx<T> acc, cpx<T> a, cpx<T> b) {
  acc.r = fma(a.r, b.r, acc.r);
  acc.r = fma(a.i, b.i, acc.r);
  acc.i = fma(a.r, b.i, acc.i);
  acc.i = fma(-a.i, b.r, acc.i);
  return acc;
}
// acc + a * conj(b)
template <class T> DSL_HD cpx<T> cmaddj(cpx<T> acc, cpx<T> a, cpx<T> b) {
  acc.r = fma(a.r, b.r, acc.r);
  acc.r = fma(a.i, b.i, acc.r);
  acc.i = fma(a.i, b.r, acc.i);
  acc.i = fma(-a.r, b.i, acc.i);
  return acc;
}
// acc + s * a (real s)
template <class T> DSL_HD cpx<T> rmadd(cpx<T> acc, T s, cpx<T> a) {
  acc.r = fma(s, a.r, acc.r);
  acc.i = fma(s, a.i, acc.i);
  return acc;
}

// ---------------------------------------------------------------- storage
struct C64 {
  using word = float2;
  using real = float;
  template <class T> static DSL_HD cpx<T> load(const word* p) {
    word w = *p;
    return {T(w.x), T(w.y)};
  }
  template <class T> static DSL_HD void store(word* p, cpx<T> v) { *p = make_float2(float(v.r), float(v.i)); }
};

struct C128 {
  using word = double2;
  using real = double;
  template <class T> static DSL_HD cpx<T> load(const word* p) {
    word w = *p;
    return {T(w.x), T(w.y)};
  }
  template <class T> static DSL_HD void store(word* p, cpx<T> v) { *p = make_double2(double(v.r), double(v.i)); }
};

DSL_HD uint32_t f32_to_bf16_rne(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0u;  // NaN stays NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}

// bf16 pair: low half = real part, high half = imaginary part
struct BF16 {
  using word = uint32_t;
  using real = float;
  template <class T> static DSL_HD cpx<T> load(const word* p) {
    word w = *p;
    return {T(__builtin_bit_cast(float, w << 16)), T(__builtin_bit_cast(float, w & 0xffff0000u))};
  }
  template <class T> static DSL_HD void store(word* p, cpx<T> v) {
    *p = f32_to_bf16_rne(float(v.r)) | (f32_to_bf16_rne(float(v.i)) << 16);
  }
};

// IEEE binary16 pair: low half = real part, high half = imaginary part
struct F16 {
  using word = uint32_t;
  using real = float;
  template <class T> static DSL_HD cpx<T> load(const word* p) {
    word w = *p;
    _Float16 re = __builtin_bit_cast(_Float16, uint16_t(w & 0xffffu));
    _Float16 im = __builtin_bit_cast(_Float16, uint16_t(w >> 16));
    return {T(float(re)), T(float(im))};
  }
  template <class T> static DSL_HD void store(word* p, cpx<T> v) {
    uint16_t re = __builtin_bit_cast(uint16_t, _Float16(float(v.r)));
    uint16_t im = __builtin_bit_cast(uint16_t, _Float16(float(v.i)));
    *p = uint32_t(re) | (uint32_t(im) << 16);
  }
};

// ---------------------------------------------------------------- fast division
// q = n / d for 0 <= n < 2^31 with a multiply-high (round-up method:
// s = ceil(log2 d), m = floor(2^32 (2^s - d) / d) + 1, q = (mulhi(n, m) + n) >> s).
struct FastDiv {
  uint32_t d, m, s;
  static FastDiv make(uint32_t d) {
    FastDiv f;
    f.d = d;
    uint32_t s = 0;
    while ((1ull << s) < d) ++s;
    f.s = s;
    f.m = uint32_t(((1ull << 32) * ((1ull << s) - d)) / d + 1);
    return f;
  }
  DSL_HD uint32_t div(uint32_t n) const {
#if defined(__HIP_DEVICE_COMPILE__)
    uint32_t hi = __umulhi(n, m);
#else
    uint32_t hi = uint32_t((uint64_t(n) * m) >> 32);
#endif
    return (hi + n) >> s;
  }
};

// ---------------------------------------------------------------- geometry
struct Geom {
  int n[4];          // Nx, Ny, Nz, Nt
  int stride[4];     // 1, Nx, Nx Ny, Nx Ny Nz
  uint32_t vol;
  int nv;
  FastDiv dx, dy, dz;
};

struct SiteNbr {
  int c[4];        // coordinates
  int fwd[4];      // s(x + mu) - s
  int bwd[4];      // s(x - mu) - s
};

DSL_HD SiteNbr site_nbr(const Geom& g, uint32_t s) {
  SiteNbr r;
  uint32_t q1 = g.dx.div(s);
  r.c[0] = int(s - q1 * uint32_t(g.n[0]));
  uint32_t q2 = g.dy.div(q1);
  r.c[1] = int(q1 - q2 * uint32_t(g.n[1]));
  uint32_t q3 = g.dz.div(q2);
  r.c[2] = int(q2 - q3 * uint32_t(g.n[2]));
  r.c[3] = int(q3);
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    const int wrap = (g.n[mu] - 1) * g.stride[mu];
    r.fwd[mu] = (r.c[mu] == g.n[mu] - 1) ? -wrap : g.stride[mu];
    r.bwd[mu] = (r.c[mu] == 0) ? wrap : -g.stride[mu];
  }
  return r;
}

// Row traversal.  A workgroup owns one chunk of `sb` consecutive sites of an
// x-row, so y, z, t and the y/z/t neighbour offsets are uniform across it.
// Rows are visited plane by plane (all chunks and y of one (z, t)), and the
// (z, t) planes in bands of `bt` time slices: t fastest inside a band, then z,
// then the next band.  A site's z- and t-neighbour rows are then at most
// bt planes away in visiting order, which keeps them inside the L2 of the XCD
// that needs them (a plain lexicographic walk puts the t-neighbours a whole
// time slice away).
struct RowTraversal {
  uint32_t sb, chunks;       // sites per chunk, chunks per x-row
  uint32_t rows_plane;       // Ny * chunks
  uint32_t bt, band_planes;  // band width in t, planes per full band (bt * Nz)
  uint32_t nbands, btlast;   // number of bands, width of the last band
  FastDiv d_plane, d_chunks, d_band, d_bt, d_btlast;
};

inline RowTraversal make_row_traversal(const Geom& g, uint32_t sb, uint32_t bt) {
  RowTraversal r;
  r.sb = sb;
  r.chunks = (uint32_t(g.n[0]) + sb - 1) / sb;
  r.rows_plane = uint32_t(g.n[1]) * r.chunks;
  if (bt < 1) bt = 1;
  if (bt > uint32_t(g.n[3])) bt = g.n[3];
  r.bt = bt;
  r.band_planes = bt * uint32_t(g.n[2]);
  r.nbands = (uint32_t(g.n[3]) + bt - 1) / bt;
  r.btlast = uint32_t(g.n[3]) - bt * (r.nbands - 1);
  r.d_plane = FastDiv::make(r.rows_plane);
  r.d_chunks = FastDiv::make(r.chunks);
  r.d_band = FastDiv::make(r.band_planes);
  r.d_bt = FastDiv::make(bt);
  r.d_btlast = FastDiv::make(r.btlast);
  return r;
}

DSL_HD SiteNbr nbr_from_coords(const Geom& g, int x, int y, int z, int t) {
  SiteNbr r;
  r.c[0] = x;
  r.c[1] = y;
  r.c[2] = z;
  r.c[3] = t;
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    const int wrap = (g.n[mu] - 1) * g.stride[mu];
    r.fwd[mu] = (r.c[mu] == g.n[mu] - 1) ? -wrap : g.stride[mu];
    r.bwd[mu] = (r.c[mu] == 0) ? wrap : -g.stride[mu];
  }
  return r;
}

// Site of lane `xi` of logical row-chunk block L; live = false past the row end.
DSL_HD SiteNbr row_site(const Geom& g, const RowTraversal& tr, uint32_t L, uint32_t xi, uint32_t& s, bool& live) {
  const uint32_t p = tr.d_plane.div(L);
  const uint32_t rin = L - p * tr.rows_plane;
  const uint32_t y = tr.d_chunks.div(rin);
  const uint32_t chunk = rin - y * tr.chunks;
  const uint32_t band = tr.d_band.div(p);
  const uint32_t q = p - band * tr.band_planes;
  const bool last = band + 1 == tr.nbands;
  const uint32_t z = last ? tr.d_btlast.div(q) : tr.d_bt.div(q);
  const uint32_t tt = q - z * (last ? tr.btlast : tr.bt);
  const uint32_t t = band * tr.bt + tt;
  const uint32_t x = chunk * tr.sb + xi;
  live = x < uint32_t(g.n[0]);
  s = x + uint32_t(g.n[0]) * (y + uint32_t(g.n[1]) * (z + uint32_t(g.n[2]) * t));
  return nbr_from_coords(g, int(x), int(y), int(z), int(t));
}

// Hardware dispatches workgroup b to XCD b % 8.  Map the first 8*floor(nb/8)
// workgroups so that XCD k receives a contiguous range of logical blocks.
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t nb, bool on = true) {
  if (!on) return b;
  const uint32_t per = nb >> 3;
  if (b < (per << 3)) return (b & 7u) * per + (b >> 3);
  return b;
}

// Output epilogues of the D_W row kernels fused for the solver (see rows.hpp):
// EPI_STORE out = result; EPI_NORM also the per-column |out|^2 sums;
// EPI_AXPY out -= alpha[v] result in place, with the |out|^2 sums.
enum { EPI_STORE = 0, EPI_NORM = 1, EPI_AXPY = 2 };

struct EpiArgs {
  const double* alpha = nullptr;  // EPI_AXPY: one coefficient per column (device)
  double* partial = nullptr;      // EPI_NORM, EPI_AXPY: [workgroups][nv] (device)
  uint32_t capacity = 0;          // workgroups the partial array holds
  uint32_t blocks = 0;            // set by the launcher: workgroups that wrote partials
};

}  // namespace dsl
