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

// Hardware dispatches workgroup b to XCD b % 8.  Map the first 8*floor(nb/8)
// workgroups so that XCD k receives a contiguous range of logical blocks.
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t nb) {
  const uint32_t per = nb >> 3;
  if (b < (per << 3)) return (b & 7u) * per + (b >> 3);
  return b;
}

}  // namespace dsl
