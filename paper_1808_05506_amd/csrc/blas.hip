// Precision conversion and the BLAS-1 kernels of the mixed-precision solver.
//
// Fields are [site][comps][nv] complex with the column (right-hand side)
// index fastest.  Per-column reductions accumulate in FP64: every thread sums
// its rows in a fixed order, the block reduces through LDS in a fixed tree,
// and a final kernel sums the kReduceBlocks block partials in a fixed order
// too, so results are bitwise reproducible run to run.  When 16 / (word
// bytes) divides nv, the kernels move 16-byte chunks (several columns per
// thread) instead of single words.
#include "launch.hpp"

namespace dsl {

template <int DT> struct StorageOf;
template <> struct StorageOf<DT_C64> { using type = C64; };
template <> struct StorageOf<DT_C128> { using type = C128; };
template <> struct StorageOf<DT_BF16> { using type = BF16; };
template <> struct StorageOf<DT_F16> { using type = F16; };

// ---------------------------------------------------------------- conversion
template <class SI, class SO, class T>
__global__ void __launch_bounds__(256) convert_kernel(const typename SI::word* __restrict__ src,
                                                      typename SO::word* __restrict__ dst, size_t n) {
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
    SO::template store<T>(dst + i, SI::template load<T>(src + i));
}

static dim3 stream_grid(size_t n) {
  size_t b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  if (b == 0) b = 1;
  return dim3(unsigned(b));
}

template <int DI, int DO>
static void convert_t(const void* src, void* dst, size_t n, hipStream_t st) {
  using SI = typename StorageOf<DI>::type;
  using SO = typename StorageOf<DO>::type;
  // FP64 arithmetic only when both ends are FP64; a narrowing store from FP64
  // rounds once, directly from the double value.
  if (DI == DT_C128 || DO == DT_C128)
    hipLaunchKernelGGL((convert_kernel<SI, SO, double>), stream_grid(n), dim3(256), 0, st,
                       (const typename SI::word*)src, (typename SO::word*)dst, n);
  else
    hipLaunchKernelGGL((convert_kernel<SI, SO, float>), stream_grid(n), dim3(256), 0, st,
                       (const typename SI::word*)src, (typename SO::word*)dst, n);
}

template <int DI>
static hipError_t convert_from(const void* src, int ddt, void* dst, size_t n, hipStream_t st) {
  switch (ddt) {
    case DT_C64: convert_t<DI, DT_C64>(src, dst, n, st); break;
    case DT_C128: convert_t<DI, DT_C128>(src, dst, n, st); break;
    case DT_BF16: convert_t<DI, DT_BF16>(src, dst, n, st); break;
    case DT_F16: convert_t<DI, DT_F16>(src, dst, n, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_convert(const void* src, int sdt, void* dst, int ddt, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  switch (sdt) {
    case DT_C64: return convert_from<DT_C64>(src, ddt, dst, n, st);
    case DT_C128: return convert_from<DT_C128>(src, ddt, dst, n, st);
    case DT_BF16: return convert_from<DT_BF16>(src, ddt, dst, n, st);
    case DT_F16: return convert_from<DT_F16>(src, ddt, dst, n, st);
  }
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------- gauge compression
// Vc[l][a][b] = V[l][a][b] for rows a = 0, 1 of every 3x3 link l (6 of its 9
// words); the third row is completed from them where the links are read.
template <class W>
__global__ void __launch_bounds__(256) compress_links_kernel(const W* __restrict__ src, W* __restrict__ dst,
                                                             size_t n) {
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x) {
    const size_t l = i / 6, e = i - l * 6;
    dst[i] = src[l * 9 + e];
  }
}

hipError_t launch_compress_links(int dtype, size_t links, const void* V, void* Vc, hipStream_t st) {
  const size_t n = links * 6;
  if (n == 0) return hipSuccess;
  switch (dtype) {
    case DT_C64:
      hipLaunchKernelGGL((compress_links_kernel<C64::word>), stream_grid(n), dim3(256), 0, st,
                         (const C64::word*)V, (C64::word*)Vc, n);
      break;
    case DT_C128:
      hipLaunchKernelGGL((compress_links_kernel<C128::word>), stream_grid(n), dim3(256), 0, st,
                         (const C128::word*)V, (C128::word*)Vc, n);
      break;
    case DT_BF16:
    case DT_F16:
      hipLaunchKernelGGL((compress_links_kernel<uint32_t>), stream_grid(n), dim3(256), 0, st, (const uint32_t*)V,
                         (uint32_t*)Vc, n);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- reductions
// Block (vc, ry): lane x = column, y = row within the block's stride.
struct ColShape {
  dim3 grid, block;
};
static ColShape col_shape(int nv) {
  const int vc = nv < 64 ? nv : 64;
  int ry = 256 / vc;
  if (ry < 1) ry = 1;
  ColShape c;
  c.block = dim3(vc, ry);
  c.grid = dim3(kReduceBlocks, (nv + vc - 1) / vc);
  return c;
}

// sum over threadIdx.y of val (per column lane), result valid in threadIdx.y == 0
__device__ __forceinline__ double block_col_sum(double val, double* sh) {
  const int vc = blockDim.x, ry = blockDim.y;
  sh[threadIdx.y * vc + threadIdx.x] = val;
  __syncthreads();
  for (int w = 1; w < ry; w <<= 1) {
    if ((threadIdx.y % (2 * w)) == 0 && threadIdx.y + w < ry)
      sh[threadIdx.y * vc + threadIdx.x] += sh[(threadIdx.y + w) * vc + threadIdx.x];
    __syncthreads();
  }
  return sh[threadIdx.x];
}

template <class S>
__global__ void __launch_bounds__(256) norm2_kernel(const typename S::word* __restrict__ x, size_t rows, int nv,
                                                    double* __restrict__ partial) {
  extern __shared__ double shd[];
  const int v = blockIdx.y * blockDim.x + threadIdx.x;
  double acc = 0.0;
  if (v < nv)
    for (size_t r = size_t(blockIdx.x) * blockDim.y + threadIdx.y; r < rows; r += size_t(gridDim.x) * blockDim.y) {
      cpx<double> z = S::template load<double>(x + r * nv + v);
      acc = fma(z.r, z.r, fma(z.i, z.i, acc));
    }
  double tot = block_col_sum(acc, shd);
  if (threadIdx.y == 0 && v < nv) partial[size_t(blockIdx.x) * nv + v] = tot;
}

// out[v] = sum over the kReduceBlocks partials of column v: one workgroup per
// column, each thread adds a fixed strided subset in index order, then a
// fixed LDS tree.
__global__ void __launch_bounds__(256) finish_sum_kernel(const double* __restrict__ partial, int nb, int nv,
                                                         double* __restrict__ out) {
  __shared__ double sh[256];
  const int v = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) s += partial[size_t(b) * nv + v];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[v] = sh[0];
}

static hipError_t finish(const double* partial, int nv, double* out, hipStream_t st) {
  hipLaunchKernelGGL(finish_sum_kernel, dim3(nv), dim3(256), 0, st, partial, kReduceBlocks, nv, out);
  return hipGetLastError();
}

// ---- 16-byte vectorised forms (used when VW = 16 / word bytes divides nv).
// Thread (cx, y) of a (nv / VW, ry) block handles the 16-byte chunks
// c = g, g + G, ... (g its global index, G the thread count, a multiple of
// nv / VW), so its VW columns cx VW .. cx VW + VW - 1 never change and
// consecutive lanes read consecutive 16 bytes.
template <class S>
struct Vec {
  using W = typename S::word;
  static constexpr int VW = 16 / int(sizeof(W));
  static __device__ __forceinline__ void unpack(u32x4 z, W (&w)[VW]) {
#pragma unroll
    for (int k = 0; k < VW; ++k) {
      if constexpr (VW == 1) {
        w[k] = __builtin_bit_cast(W, z);
      } else if constexpr (VW == 2) {
        w[k] = __builtin_bit_cast(W, u32x2{z[2 * k], z[2 * k + 1]});
      } else {
        // 4-byte words are uint32_t: plain element reads (a bit cast of a
        // vector element is miscompiled by this compiler: it reads element 0)
        static_assert(__is_same(W, uint32_t), "4-byte storage words are uint32_t");
        w[k] = z[k];
      }
    }
  }
  static __device__ __forceinline__ u32x4 pack(const W (&w)[VW]) {
    u32x4 z;
#pragma unroll
    for (int k = 0; k < VW; ++k) {
      if constexpr (VW == 1) {
        z = __builtin_bit_cast(u32x4, w[k]);
      } else if constexpr (VW == 2) {
        const u32x2 a = __builtin_bit_cast(u32x2, w[k]);
        z[2 * k] = a[0];
        z[2 * k + 1] = a[1];
      } else {
        z[k] = w[k];
      }
    }
    return z;
  }
};

// VW per-column accumulators of each thread summed over threadIdx.y, written
// as the block's partial of columns cx VW + k.
template <int VW>
__device__ __forceinline__ void vec_block_partial(const double (&acc)[VW], double* sh, double* partial, int nv) {
  const int cols = blockDim.x, ry = blockDim.y;
#pragma unroll
  for (int k = 0; k < VW; ++k) {
    sh[threadIdx.y * cols + threadIdx.x] = acc[k];
    __syncthreads();
    for (int w = 1; w < ry; w <<= 1) {
      if ((threadIdx.y % (2 * w)) == 0 && threadIdx.y + w < ry)
        sh[threadIdx.y * cols + threadIdx.x] += sh[(threadIdx.y + w) * cols + threadIdx.x];
      __syncthreads();
    }
    if (threadIdx.y == 0) partial[size_t(blockIdx.x) * nv + threadIdx.x * VW + k] = sh[threadIdx.x];
    __syncthreads();
  }
}

template <class S>
__global__ void __launch_bounds__(256) norm2_vec_kernel(const u32x4* __restrict__ x, size_t chunks, int nv,
                                                        double* __restrict__ partial) {
  using W = typename S::word;
  constexpr int VW = Vec<S>::VW;
  extern __shared__ double shd[];
  const size_t G = size_t(gridDim.x) * blockDim.x * blockDim.y;
  const size_t g0 = (size_t(blockIdx.x) * blockDim.y + threadIdx.y) * blockDim.x + threadIdx.x;
  double acc[VW];
#pragma unroll
  for (int k = 0; k < VW; ++k) acc[k] = 0.0;
  // four independent chunks in flight per thread
  for (size_t c = g0; c < chunks; c += 4 * G) {
    u32x4 z[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const size_t cu = c + u * G;
      z[u] = x[cu < chunks ? cu : c];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (c + u * G < chunks) {
        W w[VW];
        Vec<S>::unpack(z[u], w);
#pragma unroll
        for (int k = 0; k < VW; ++k) {
          const cpx<double> q = S::template load<double>(&w[k]);
          acc[k] = fma(q.r, q.r, fma(q.i, q.i, acc[k]));
        }
      }
    }
  }
  vec_block_partial<VW>(acc, shd, partial, nv);
}

template <class S>
static bool vec_ok(int nv, const void* p) {
  return nv % Vec<S>::VW == 0 && (reinterpret_cast<uintptr_t>(p) & 15) == 0;
}

template <class S>
static void norm2_vec(const void* x, size_t n, int nv, double* partial, hipStream_t st) {
  const int cols = nv / Vec<S>::VW;
  const int ry = 256 / cols > 0 ? 256 / cols : 1;
  const size_t lds = size_t(cols) * ry * sizeof(double);
  hipLaunchKernelGGL(norm2_vec_kernel<S>, dim3(kReduceBlocks), dim3(cols, ry), lds, st, (const u32x4*)x,
                     n / Vec<S>::VW, nv, partial);
}

hipError_t launch_norm2(int dtype, const void* x, size_t sites, int comps, int nv, double* partial, double* out,
                        hipStream_t st) {
  const ColShape c = col_shape(nv);
  const size_t rows = sites * comps;
  const size_t n = rows * nv;
  const size_t lds = size_t(c.block.x) * c.block.y * sizeof(double);
  switch (dtype) {
    case DT_C64:
      if (nv <= 512 && vec_ok<C64>(nv, x)) norm2_vec<C64>(x, n, nv, partial, st);
      else hipLaunchKernelGGL(norm2_kernel<C64>, c.grid, c.block, lds, st, (const float2*)x, rows, nv, partial);
      break;
    case DT_C128:
      if (nv <= 256 && vec_ok<C128>(nv, x)) norm2_vec<C128>(x, n, nv, partial, st);
      else hipLaunchKernelGGL(norm2_kernel<C128>, c.grid, c.block, lds, st, (const double2*)x, rows, nv, partial);
      break;
    case DT_BF16:
      if (nv <= 1024 && vec_ok<BF16>(nv, x)) norm2_vec<BF16>(x, n, nv, partial, st);
      else hipLaunchKernelGGL(norm2_kernel<BF16>, c.grid, c.block, lds, st, (const uint32_t*)x, rows, nv, partial);
      break;
    case DT_F16:
      if (nv <= 1024 && vec_ok<F16>(nv, x)) norm2_vec<F16>(x, n, nv, partial, st);
      else hipLaunchKernelGGL(norm2_kernel<F16>, c.grid, c.block, lds, st, (const uint32_t*)x, rows, nv, partial);
      break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return finish(partial, nv, out, st);
}

// ---------------------------------------------------------------- elementwise
__global__ void __launch_bounds__(256) xmy_kernel(const double2* __restrict__ b, const double2* __restrict__ t,
                                                  double2* __restrict__ r, size_t n) {
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x) {
    double2 x = b[i], y = t[i];
    r[i] = make_double2(x.x - y.x, x.y - y.y);
  }
}

hipError_t launch_xmy(const void* b, const void* t, void* r, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(xmy_kernel, stream_grid(n), dim3(256), 0, st, (const double2*)b, (const double2*)t,
                     (double2*)r, n);
  return hipGetLastError();
}

template <class S>
__global__ void __launch_bounds__(256) scale_to_kernel(const double2* __restrict__ hi, typename S::word* __restrict__ lo,
                                                       const double* __restrict__ inv, size_t n, int nv) {
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x) {
    const double s = inv[i % nv];
    double2 x = hi[i];
    S::template store<double>(lo + i, cpx<double>{s * x.x, s * x.y});
  }
}

template <class S>
__global__ void __launch_bounds__(256) axpy_promote_kernel(double2* __restrict__ x, const typename S::word* __restrict__ e,
                                                           const double* __restrict__ sc, size_t n, int nv) {
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x) {
    const double s = sc[i % nv];
    cpx<double> z = S::template load<double>(e + i);
    double2 y = x[i];
    x[i] = make_double2(fma(s, z.r, y.x), fma(s, z.i, y.y));
  }
}

hipError_t launch_scale_to(const void* hi, int lodt, void* lo, const double* inv, size_t sites, int comps, int nv,
                           hipStream_t st) {
  const size_t n = sites * comps * nv;
  const dim3 gr = stream_grid(n), bl(256);
  switch (lodt) {
    case DT_C64: hipLaunchKernelGGL(scale_to_kernel<C64>, gr, bl, 0, st, (const double2*)hi, (float2*)lo, inv, n, nv); break;
    case DT_BF16: hipLaunchKernelGGL(scale_to_kernel<BF16>, gr, bl, 0, st, (const double2*)hi, (uint32_t*)lo, inv, n, nv); break;
    case DT_F16: hipLaunchKernelGGL(scale_to_kernel<F16>, gr, bl, 0, st, (const double2*)hi, (uint32_t*)lo, inv, n, nv); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_axpy_promote(void* x, int lodt, const void* e, const double* s, size_t sites, int comps, int nv,
                               hipStream_t st) {
  const size_t n = sites * comps * nv;
  const dim3 gr = stream_grid(n), bl(256);
  switch (lodt) {
    case DT_C64: hipLaunchKernelGGL(axpy_promote_kernel<C64>, gr, bl, 0, st, (double2*)x, (const float2*)e, s, n, nv); break;
    case DT_BF16: hipLaunchKernelGGL(axpy_promote_kernel<BF16>, gr, bl, 0, st, (double2*)x, (const uint32_t*)e, s, n, nv); break;
    case DT_F16: hipLaunchKernelGGL(axpy_promote_kernel<F16>, gr, bl, 0, st, (double2*)x, (const uint32_t*)e, s, n, nv); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// e += alpha p; r -= alpha q; per-column |r|^2 partials (FP32 arithmetic for the
// updates, FP64 for the norm)
// XE = false: the residual update alone (e and p unused).
template <class S, bool XE = true>
__global__ void __launch_bounds__(256) cg_update_xr_kernel(typename S::word* __restrict__ e, typename S::word* __restrict__ r,
                                                           const typename S::word* __restrict__ p,
                                                           const typename S::word* __restrict__ q,
                                                           const double* __restrict__ alpha, size_t rows, int nv,
                                                           double* __restrict__ partial) {
  extern __shared__ double shd[];
  const int v = blockIdx.y * blockDim.x + threadIdx.x;
  double acc = 0.0;
  if (v < nv) {
    const float a = float(alpha[v]);
    for (size_t row = size_t(blockIdx.x) * blockDim.y + threadIdx.y; row < rows; row += size_t(gridDim.x) * blockDim.y) {
      const size_t i = row * nv + v;
      if constexpr (XE) {
        cpx<float> ev = S::template load<float>(e + i), pv = S::template load<float>(p + i);
        S::template store<float>(e + i, rmadd(ev, a, pv));
      }
      cpx<float> rv = S::template load<float>(r + i), qv = S::template load<float>(q + i);
      rv = rmadd(rv, -a, qv);
      S::template store<float>(r + i, rv);
      cpx<double> rs = S::template load<double>(r + i);  // the stored (rounded) residual
      acc = fma(rs.r, rs.r, fma(rs.i, rs.i, acc));
    }
  }
  double tot = block_col_sum(acc, shd);
  if (threadIdx.y == 0 && v < nv) partial[size_t(blockIdx.x) * nv + v] = tot;
}

// Vectorised e += alpha p; r -= alpha q with the |r|^2 partials of the stored
// (rounded) residual.
template <class S, bool XE = true>
__global__ void __launch_bounds__(256) cg_update_xr_vec_kernel(u32x4* __restrict__ e, u32x4* __restrict__ r,
                                                               const u32x4* __restrict__ p,
                                                               const u32x4* __restrict__ q,
                                                               const double* __restrict__ alpha, size_t chunks, int nv,
                                                               double* __restrict__ partial) {
  using W = typename S::word;
  constexpr int VW = Vec<S>::VW;
  extern __shared__ double shd[];
  const size_t G = size_t(gridDim.x) * blockDim.x * blockDim.y;
  const size_t g0 = (size_t(blockIdx.x) * blockDim.y + threadIdx.y) * blockDim.x + threadIdx.x;
  float a[VW];
  double acc[VW];
#pragma unroll
  for (int k = 0; k < VW; ++k) {
    a[k] = float(alpha[threadIdx.x * VW + k]);
    acc[k] = 0.0;
  }
  for (size_t c = g0; c < chunks; c += 2 * G) {
    u32x4 ze[2], zp[2], zr[2], zq[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const size_t cu = c + u * G < chunks ? c + u * G : c;
      if constexpr (XE) {
        ze[u] = e[cu];
        zp[u] = p[cu];
      }
      zr[u] = r[cu];
      zq[u] = q[cu];
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      if (c + u * G < chunks) {
        W wr[VW], wq[VW];
        if constexpr (XE) {
          W we[VW], wp[VW];
          Vec<S>::unpack(ze[u], we);
          Vec<S>::unpack(zp[u], wp);
#pragma unroll
          for (int k = 0; k < VW; ++k)
            S::template store<float>(&we[k], rmadd(S::template load<float>(&we[k]), a[k], S::template load<float>(&wp[k])));
          e[c + u * G] = Vec<S>::pack(we);
        }
        Vec<S>::unpack(zr[u], wr);
        Vec<S>::unpack(zq[u], wq);
#pragma unroll
        for (int k = 0; k < VW; ++k) {
          S::template store<float>(&wr[k], rmadd(S::template load<float>(&wr[k]), -a[k], S::template load<float>(&wq[k])));
          const cpx<double> rs = S::template load<double>(&wr[k]);
          acc[k] = fma(rs.r, rs.r, fma(rs.i, rs.i, acc[k]));
        }
        r[c + u * G] = Vec<S>::pack(wr);
      }
    }
  }
  vec_block_partial<VW>(acc, shd, partial, nv);
}

template <class S, bool XE = true>
static void cg_update_xr_vec(void* e, void* r, const void* p, const void* q, const double* alpha, size_t n, int nv,
                             double* partial, hipStream_t st) {
  const int cols = nv / Vec<S>::VW;
  const int ry = 256 / cols > 0 ? 256 / cols : 1;
  const size_t lds = size_t(cols) * ry * sizeof(double);
  hipLaunchKernelGGL((cg_update_xr_vec_kernel<S, XE>), dim3(kReduceBlocks), dim3(cols, ry), lds, st, (u32x4*)e, (u32x4*)r,
                     (const u32x4*)p, (const u32x4*)q, alpha, n / Vec<S>::VW, nv, partial);
}

template <class S>
static bool vec_ok4(int nv, const void* a, const void* b, const void* c, const void* d) {
  return vec_ok<S>(nv, a) && vec_ok<S>(nv, b) && vec_ok<S>(nv, c) && vec_ok<S>(nv, d) &&
         nv / Vec<S>::VW <= 256;
}

hipError_t launch_cg_update_xr(int dtype, void* e, void* r, const void* p, const void* q, const double* alpha,
                               size_t sites, int comps, int nv, double* partial, double* out, hipStream_t st) {
  const ColShape c = col_shape(nv);
  const size_t rows = sites * comps;
  const size_t lds = size_t(c.block.x) * c.block.y * sizeof(double);
  const size_t n = rows * nv;
  switch (dtype) {
    case DT_C64:
      if (vec_ok4<C64>(nv, e, r, p, q)) cg_update_xr_vec<C64>(e, r, p, q, alpha, n, nv, partial, st);
      else
        hipLaunchKernelGGL(cg_update_xr_kernel<C64>, c.grid, c.block, lds, st, (float2*)e, (float2*)r,
                           (const float2*)p, (const float2*)q, alpha, rows, nv, partial);
      break;
    case DT_BF16:
      if (vec_ok4<BF16>(nv, e, r, p, q)) cg_update_xr_vec<BF16>(e, r, p, q, alpha, n, nv, partial, st);
      else
        hipLaunchKernelGGL(cg_update_xr_kernel<BF16>, c.grid, c.block, lds, st, (uint32_t*)e, (uint32_t*)r,
                           (const uint32_t*)p, (const uint32_t*)q, alpha, rows, nv, partial);
      break;
    case DT_F16:
      if (vec_ok4<F16>(nv, e, r, p, q)) cg_update_xr_vec<F16>(e, r, p, q, alpha, n, nv, partial, st);
      else
        hipLaunchKernelGGL(cg_update_xr_kernel<F16>, c.grid, c.block, lds, st, (uint32_t*)e, (uint32_t*)r,
                           (const uint32_t*)p, (const uint32_t*)q, alpha, rows, nv, partial);
      break;
    default: return hipErrorInvalidValue;
  }
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  return finish(partial, nv, out, st);
}

template <class S>
__global__ void __launch_bounds__(256) cg_update_p_kernel(typename S::word* __restrict__ p,
                                                          const typename S::word* __restrict__ r,
                                                          const double* __restrict__ beta, size_t n, int nv) {
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x) {
    const float b = float(beta[i % nv]);
    cpx<float> pv = S::template load<float>(p + i), rv = S::template load<float>(r + i);
    S::template store<float>(p + i, rmadd(rv, b, pv));
  }
}

hipError_t launch_cg_update_p(int dtype, void* p, const void* r, const double* beta, size_t sites, int comps, int nv,
                              hipStream_t st) {
  const size_t n = sites * comps * nv;
  const dim3 gr = stream_grid(n), bl(256);
  switch (dtype) {
    case DT_C64: hipLaunchKernelGGL(cg_update_p_kernel<C64>, gr, bl, 0, st, (float2*)p, (const float2*)r, beta, n, nv); break;
    case DT_BF16: hipLaunchKernelGGL(cg_update_p_kernel<BF16>, gr, bl, 0, st, (uint32_t*)p, (const uint32_t*)r, beta, n, nv); break;
    case DT_F16: hipLaunchKernelGGL(cg_update_p_kernel<F16>, gr, bl, 0, st, (uint32_t*)p, (const uint32_t*)r, beta, n, nv); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class S>
static hipError_t update_r_t(void* r, const void* s_, const double* alpha, size_t rows, int nv, double* partial,
                             hipStream_t st) {
  using W = typename S::word;
  if (vec_ok<S>(nv, r) && vec_ok<S>(nv, s_) && nv / Vec<S>::VW <= 256) {
    cg_update_xr_vec<S, false>(nullptr, r, nullptr, s_, alpha, rows * nv, nv, partial, st);
  } else {
    const ColShape c = col_shape(nv);
    const size_t lds = size_t(c.block.x) * c.block.y * sizeof(double);
    hipLaunchKernelGGL((cg_update_xr_kernel<S, false>), c.grid, c.block, lds, st, (W*)nullptr, (W*)r,
                       (const W*)nullptr, (const W*)s_, alpha, rows, nv, partial);
  }
  return hipGetLastError();
}

hipError_t launch_cg_update_r(int dtype, void* r, const void* s_, const double* alpha, size_t sites, int comps, int nv,
                              double* partial, double* out, hipStream_t st) {
  const size_t rows = sites * comps;
  hipError_t err;
  switch (dtype) {
    case DT_C64: err = update_r_t<C64>(r, s_, alpha, rows, nv, partial, st); break;
    case DT_BF16: err = update_r_t<BF16>(r, s_, alpha, rows, nv, partial, st); break;
    case DT_F16: err = update_r_t<F16>(r, s_, alpha, rows, nv, partial, st); break;
    default: return hipErrorInvalidValue;
  }
  if (err != hipSuccess) return err;
  return finish(partial, nv, out, st);
}

// e += alpha[v] p;  p = r + beta[v] p  (the old p in both), FP32 arithmetic.
// Vectorised: thread (cx, y) of a (nv / VW, ry) block keeps the columns
// cx VW .. cx VW + VW - 1 (as in the reductions).
template <class S, bool NT = false>
__global__ void __launch_bounds__(256) cg_update_ep_vec_kernel(u32x4* __restrict__ e, u32x4* __restrict__ p,
                                                               const u32x4* __restrict__ r,
                                                               const double* __restrict__ alpha,
                                                               const double* __restrict__ beta, size_t chunks) {
  using W = typename S::word;
  constexpr int VW = Vec<S>::VW;
  const size_t G = size_t(gridDim.x) * blockDim.x * blockDim.y;
  const size_t g0 = (size_t(blockIdx.x) * blockDim.y + threadIdx.y) * blockDim.x + threadIdx.x;
  float a[VW], b[VW];
#pragma unroll
  for (int k = 0; k < VW; ++k) {
    a[k] = float(alpha[threadIdx.x * VW + k]);
    b[k] = float(beta[threadIdx.x * VW + k]);
  }
  for (size_t c = g0; c < chunks; c += G) {
    W we[VW], wp[VW], wr[VW];
    if constexpr (NT) {
      Vec<S>::unpack(__builtin_nontemporal_load(&e[c]), we);
      Vec<S>::unpack(__builtin_nontemporal_load(&p[c]), wp);
      Vec<S>::unpack(__builtin_nontemporal_load(&r[c]), wr);
    } else {
      Vec<S>::unpack(e[c], we);
      Vec<S>::unpack(p[c], wp);
      Vec<S>::unpack(r[c], wr);
    }
#pragma unroll
    for (int k = 0; k < VW; ++k) {
      const cpx<float> pv = S::template load<float>(&wp[k]);
      S::template store<float>(&we[k], rmadd(S::template load<float>(&we[k]), a[k], pv));
      S::template store<float>(&wp[k], rmadd(S::template load<float>(&wr[k]), b[k], pv));
    }
    if constexpr (NT) {
      __builtin_nontemporal_store(Vec<S>::pack(we), &e[c]);
      __builtin_nontemporal_store(Vec<S>::pack(wp), &p[c]);
    } else {
      e[c] = Vec<S>::pack(we);
      p[c] = Vec<S>::pack(wp);
    }
  }
}

template <class S>
__global__ void __launch_bounds__(256) cg_update_ep_kernel(typename S::word* __restrict__ e,
                                                           typename S::word* __restrict__ p,
                                                           const typename S::word* __restrict__ r,
                                                           const double* __restrict__ alpha,
                                                           const double* __restrict__ beta, size_t n, int nv) {
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x) {
    const int v = int(i % nv);
    const float a = float(alpha[v]), b = float(beta[v]);
    const cpx<float> pv = S::template load<float>(p + i);
    S::template store<float>(e + i, rmadd(S::template load<float>(e + i), a, pv));
    S::template store<float>(p + i, rmadd(S::template load<float>(r + i), b, pv));
  }
}

template <class S>
static hipError_t update_ep_t(void* e, void* p, const void* r, const double* alpha, const double* beta, size_t n,
                              int nv, hipStream_t st) {
  using W = typename S::word;
  if (vec_ok<S>(nv, e) && vec_ok<S>(nv, p) && vec_ok<S>(nv, r) && nv / Vec<S>::VW <= 256) {
    const int cols = nv / Vec<S>::VW;
    const int ry = 256 / cols > 0 ? 256 / cols : 1;
    const size_t chunks = n / Vec<S>::VW;
    size_t blocks = (chunks + size_t(cols) * ry - 1) / (size_t(cols) * ry);
    if (blocks > 8192) blocks = 8192;
    if (blocks == 0) blocks = 1;
    // non-temporal loads and stores for FP32 words (DSLASH_BLAS_NT overrides):
    // on 32^3 x 64, N_v = 12 the full-lattice update took 2508 against 2674 us
    // with them in C64, but 1412 against 1249 us in BF16 and FP16
    if (knobs().blas_nt.get(sizeof(W) == 8 ? 1 : 0))
      hipLaunchKernelGGL((cg_update_ep_vec_kernel<S, true>), dim3(unsigned(blocks)), dim3(cols, ry), 0, st,
                         (u32x4*)e, (u32x4*)p, (const u32x4*)r, alpha, beta, chunks);
    else
      hipLaunchKernelGGL((cg_update_ep_vec_kernel<S, false>), dim3(unsigned(blocks)), dim3(cols, ry), 0, st,
                         (u32x4*)e, (u32x4*)p, (const u32x4*)r, alpha, beta, chunks);
  } else {
    hipLaunchKernelGGL(cg_update_ep_kernel<S>, stream_grid(n), dim3(256), 0, st, (W*)e, (W*)p, (const W*)r, alpha,
                       beta, n, nv);
  }
  return hipGetLastError();
}

hipError_t launch_cg_update_ep(int dtype, void* e, void* p, const void* r, const double* alpha, const double* beta,
                               size_t sites, int comps, int nv, hipStream_t st) {
  const size_t n = sites * comps * nv;
  switch (dtype) {
    case DT_C64: return update_ep_t<C64>(e, p, r, alpha, beta, n, nv, st);
    case DT_BF16: return update_ep_t<BF16>(e, p, r, alpha, beta, n, nv, st);
    case DT_F16: return update_ep_t<F16>(e, p, r, alpha, beta, n, nv, st);
    default: return hipErrorInvalidValue;
  }
}

// fold[b][v] = sum of partial[i][v] over the rows i of chunk b (chunks of
// ceil(nb / kReduceBlocks) consecutive rows), in a fixed order: thread (v, y)
// adds rows y, y + ry, ... of the chunk, then a fixed LDS tree over y.
__global__ void __launch_bounds__(256) fold_rows_kernel(const double* __restrict__ partial, int nb, int nv,
                                                        int chunk, double* __restrict__ fold) {
  extern __shared__ double shd[];
  const int v = blockIdx.y * blockDim.x + threadIdx.x;
  const int r0 = blockIdx.x * chunk, r1 = r0 + chunk < nb ? r0 + chunk : nb;
  double acc = 0.0;
  if (v < nv)
    for (int r = r0 + int(threadIdx.y); r < r1; r += blockDim.y) acc += partial[size_t(r) * nv + v];
  double tot = block_col_sum(acc, shd);
  if (threadIdx.y == 0 && v < nv) fold[size_t(blockIdx.x) * nv + v] = tot;
}

hipError_t launch_finish_sum(const double* partial, int nb, int nv, double* out, double* fold, hipStream_t st) {
  if (nb > 2 * kReduceBlocks && fold) {
    const ColShape c = col_shape(nv);
    const size_t lds = size_t(c.block.x) * c.block.y * sizeof(double);
    const int chunk = (nb + kReduceBlocks - 1) / kReduceBlocks;
    hipLaunchKernelGGL(fold_rows_kernel, c.grid, c.block, lds, st, partial, nb, nv, chunk, fold);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    partial = fold;
    nb = kReduceBlocks;
  }
  hipLaunchKernelGGL(finish_sum_kernel, dim3(nv), dim3(256), 0, st, partial, nb, nv, out);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256) zero_kernel(uint32_t* __restrict__ x, size_t nwords) {
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < nwords; i += size_t(gridDim.x) * blockDim.x)
    x[i] = 0u;
}

hipError_t launch_zero(int dtype, void* x, size_t n, hipStream_t st) {
  const size_t nwords = n * dtype_bytes(dtype) / 4;
  if (nwords == 0) return hipSuccess;
  hipLaunchKernelGGL(zero_kernel, stream_grid(nwords), dim3(256), 0, st, (uint32_t*)x, nwords);
  return hipGetLastError();
}

__global__ void cg_scalars_kernel(int mode, int nv, double* rr, double* rr_new, double* pq, double* rr0,
                                  double* alpha, double* beta, double* active, double tol) {
  for (int v = threadIdx.x; v < nv; v += blockDim.x) {
    const bool on = active[v] != 0.0;
    if (mode == 0) {
      alpha[v] = (on && pq[v] > 0.0) ? rr[v] / pq[v] : 0.0;
    } else {
      beta[v] = (on && rr[v] > 0.0) ? rr_new[v] / rr[v] : 0.0;
      if (on) rr[v] = rr_new[v];
      const bool still = on && rr0[v] > 0.0 && sqrt(rr[v] / rr0[v]) > tol;
      active[v] = still ? 1.0 : 0.0;
    }
  }
}

hipError_t launch_cg_scalars(int mode, int nv, double* rr, double* rr_new, double* pq, double* rr0, double* alpha,
                             double* beta, double* active, double tol, hipStream_t st) {
  hipLaunchKernelGGL(cg_scalars_kernel, dim3(1), dim3(256), 0, st, mode, nv, rr, rr_new, pq, rr0, alpha, beta,
                     active, tol);
  return hipGetLastError();
}

}  // namespace dsl
