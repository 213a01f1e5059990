// FP32 throughput of gfx950's vector and matrix units on the D_B contraction.
//
// D_B's arithmetic is dominated, per site, hop d and right-hand side, by the
// 3 x 3 complex link times the four colour vectors of the hopped spinor (Sec. 5,
// the products W_d(x) psi(x + d) of the 80 hops).  Two ways to run it:
//
//   valu  one lane per (site, v): chi_q = W' psi_q for the four spins q, 36
//         complex multiply-adds (144 FMA), W' read from LDS (the same word for
//         the 12 lanes of a site), psi_q from LDS.
//   mfma  the same lanes, the product as 4 x 4 x 1 16-block matrix FMAs: block
//         b = four lanes (one site, v = 4j .. 4j + 3); the complex product in
//         the real 6 x 6 form [[Re W, -Im W], [Im W, Re W]] acting on
//         (Re psi, Im psi), rows split into two 4-row blocks (Re c0 c1 c2,
//         Im c0 | Im c1 c2, two zero rows), K = 6 (colour x re/im): 48 matrix
//         instructions per hop and wave.  The B operand is the lane's own psi
//         component and D row i lands in register i of the lane's own column,
//         so the (site, v) lane layout of the row-staged kernels is kept; the
//         lane builds its A row (its colour row of W', re/im arranged) from LDS.
//
// Both run NDIR = 80 hops per lane on LDS-resident data (no HBM traffic), over
// 16-site x 12-rhs workgroups; the kernels are checked against each other.
// Also measured: the raw rate of each unit on independent chains, and both in
// one instruction stream (whether matrix and vector FP32 work overlap).
//
// Build (done by the package build):
//   hipcc -x hip --offload-arch=gfx950 -O3 -Xclang -target-feature -Xclang -packed-fp32-ops fp32_contraction.hip -o fp32_contraction
// Run: ./fp32_contraction  (one GPU; prints one line per kernel)
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <vector>

typedef float f4 __attribute__((ext_vector_type(4)));

#define CK(x)                                                                        \
  do {                                                                               \
    hipError_t e_ = (x);                                                             \
    if (e_ != hipSuccess) {                                                          \
      fprintf(stderr, "HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
      exit(1);                                                                       \
    }                                                                                \
  } while (0)

namespace {

constexpr int NV = 12, R = 16, THREADS = NV * R, NDIR = 80, WSLOTS = 8;
constexpr int PSI_FLOATS = R * 12 * NV * 2;     // [site][spin*3 + colour][v] complex
constexpr int W_FLOATS = WSLOTS * R * 9 * 2;    // [slot][site][3][3] complex

struct c32 {
  float r, i;
};

__device__ __forceinline__ c32 cmadd(c32 a, c32 b, c32 c) {  // a + b c
  a.r = fmaf(b.r, c.r, a.r);
  a.r = fmaf(-b.i, c.i, a.r);
  a.i = fmaf(b.r, c.i, a.i);
  a.i = fmaf(b.i, c.r, a.i);
  return a;
}

__device__ void fill_lds(const float* __restrict__ gpsi, const float* __restrict__ gw, float* psi, float* w) {
  for (int k = threadIdx.x; k < PSI_FLOATS; k += THREADS) psi[k] = gpsi[k];
  for (int k = threadIdx.x; k < W_FLOATS; k += THREADS) w[k] = gw[k];
  __syncthreads();
}

// hop d of lane (xl, v): neighbour site (xl + d) mod R, link slot d mod 8 of the
// own site, the adjoint on odd d (as half of D_B's hops take W_{-d}(x + d)^dag)
__device__ __forceinline__ int hop_site(int xl, int d) { return (xl + d) & (R - 1); }

__global__ void __launch_bounds__(THREADS) valu_kernel(const float* __restrict__ gpsi, const float* __restrict__ gw,
                                                       float* __restrict__ out, int ndir) {
  __shared__ float psi[PSI_FLOATS];
  __shared__ float w[W_FLOATS];
  fill_lds(gpsi, gw, psi, w);
  const int v = threadIdx.x % NV, xl = threadIdx.x / NV;
  c32 acc[4][3];
  for (int q = 0; q < 4; ++q)
    for (int c = 0; c < 3; ++c) acc[q][c] = c32{0.f, 0.f};
#pragma unroll 2
  for (int d = 0; d < ndir; ++d) {
    const c32* lk = reinterpret_cast<const c32*>(w) + ((d % WSLOTS) * R + xl) * 9;
    const c32* ps = reinterpret_cast<const c32*>(psi) + hop_site(xl, d) * 12 * NV;
    const bool dag = __builtin_amdgcn_readfirstlane(d) & 1;
    c32 u[3][3], p[4][3];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        const c32 l = lk[dag ? b * 3 + a : a * 3 + b];
        u[a][b] = c32{l.r, dag ? -l.i : l.i};
      }
    for (int q = 0; q < 4; ++q)
      for (int b = 0; b < 3; ++b) p[q][b] = ps[(q * 3 + b) * NV + v];
    for (int q = 0; q < 4; ++q)
      for (int c = 0; c < 3; ++c)
        for (int b = 0; b < 3; ++b) acc[q][c] = cmadd(acc[q][c], u[c][b], p[q][b]);
  }
  float* o = out + (size_t(blockIdx.x) * THREADS + threadIdx.x) * 24;
  for (int q = 0; q < 4; ++q)
    for (int c = 0; c < 3; ++c) {
      o[(q * 3 + c) * 2] = acc[q][c].r;
      o[(q * 3 + c) * 2 + 1] = acc[q][c].i;
    }
}

__global__ void __launch_bounds__(THREADS) mfma_kernel(const float* __restrict__ gpsi, const float* __restrict__ gw,
                                                       float* __restrict__ out, int ndir) {
  __shared__ float psi[PSI_FLOATS];
  __shared__ float w[W_FLOATS];
  fill_lds(gpsi, gw, psi, w);
  const int v = threadIdx.x % NV, xl = threadIdx.x / NV, i = threadIdx.x & 3;
  // A rows of the lane: block 0 row i = Re c_i (i < 3) or Im c_0 (i = 3);
  // block 1 row i = Im c_{i+1} (i < 2) or zero
  const int a0 = i < 3 ? i : 0, a1 = i < 2 ? i + 1 : 0;
  const bool im0 = i == 3, zero1 = i >= 2;
  f4 d0[4], d1[4];
  for (int q = 0; q < 4; ++q) d0[q] = d1[q] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
  for (int d = 0; d < ndir; ++d) {
    const c32* lk = reinterpret_cast<const c32*>(w) + ((d % WSLOTS) * R + xl) * 9;
    const c32* ps = reinterpret_cast<const c32*>(psi) + hop_site(xl, d) * 12 * NV;
    const bool dag = __builtin_amdgcn_readfirstlane(d) & 1;
    float ar0[3], ai0[3], ar1[3], ai1[3];
    for (int b = 0; b < 3; ++b) {
      c32 l0 = lk[dag ? b * 3 + a0 : a0 * 3 + b], l1 = lk[dag ? b * 3 + a1 : a1 * 3 + b];
      if (dag) {
        l0.i = -l0.i;
        l1.i = -l1.i;
      }
      // Re row: (Re W, -Im W); Im row: (Im W, Re W)
      ar0[b] = im0 ? l0.i : l0.r;
      ai0[b] = im0 ? l0.r : -l0.i;
      ar1[b] = zero1 ? 0.f : l1.i;
      ai1[b] = zero1 ? 0.f : l1.r;
    }
    for (int q = 0; q < 4; ++q)
      for (int b = 0; b < 3; ++b) {
        const c32 p = ps[(q * 3 + b) * NV + v];
        d0[q] = __builtin_amdgcn_mfma_f32_4x4x1f32(ar0[b], p.r, d0[q], 0, 0, 0);
        d0[q] = __builtin_amdgcn_mfma_f32_4x4x1f32(ai0[b], p.i, d0[q], 0, 0, 0);
        d1[q] = __builtin_amdgcn_mfma_f32_4x4x1f32(ar1[b], p.r, d1[q], 0, 0, 0);
        d1[q] = __builtin_amdgcn_mfma_f32_4x4x1f32(ai1[b], p.i, d1[q], 0, 0, 0);
      }
  }
  // the lane's column: Re c0 c1 c2 = d0[q][0..2], Im c0 = d0[q][3], Im c1 c2 = d1[q][0..1]
  float* o = out + (size_t(blockIdx.x) * THREADS + threadIdx.x) * 24;
  for (int q = 0; q < 4; ++q) {
    const float re[3] = {d0[q][0], d0[q][1], d0[q][2]}, im[3] = {d0[q][3], d1[q][0], d1[q][1]};
    for (int c = 0; c < 3; ++c) {
      o[(q * 3 + c) * 2] = re[c];
      o[(q * 3 + c) * 2 + 1] = im[c];
    }
  }
}

// raw rates: ITER x 8 independent accumulators per wave
__global__ void __launch_bounds__(256) rate_mfma(float* out, int iters, float s) {
  const float a = s * threadIdx.x, b = s + threadIdx.x;
  f4 c[8];
  for (int k = 0; k < 8; ++k) c[k] = f4{0.f, 0.f, 0.f, 0.f};
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int k = 0; k < 8; ++k) c[k] = __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c[k], 0, 0, 0);
  float t = 0.f;
  for (int k = 0; k < 8; ++k) t += c[k][0] + c[k][1] + c[k][2] + c[k][3];
  out[blockIdx.x * blockDim.x + threadIdx.x] = t;
}

template <int NF>
__global__ void __launch_bounds__(256) rate_valu(float* out, int iters, float s) {
  float x[8];
  for (int k = 0; k < 8; ++k) x[k] = s * (threadIdx.x + k);
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int k = 0; k < 8; ++k)
#pragma unroll
      for (int f = 0; f < NF / 8; ++f) x[(k + f) % 8] = fmaf(x[(k + f) % 8], 0.999f, 1e-3f);
  float t = 0.f;
  for (int k = 0; k < 8; ++k) t += x[k];
  out[blockIdx.x * blockDim.x + threadIdx.x] = t;
}

// one instruction stream: per iteration 8 matrix FMAs and NF vector FMAs on
// independent data
template <int NF>
__global__ void __launch_bounds__(256) rate_both(float* out, int iters, float s) {
  const float a = s * threadIdx.x, b = s + threadIdx.x;
  f4 c[8];
  float x[8];
  for (int k = 0; k < 8; ++k) {
    c[k] = f4{0.f, 0.f, 0.f, 0.f};
    x[k] = s * (threadIdx.x + k);
  }
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      c[k] = __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c[k], 0, 0, 0);
#pragma unroll
      for (int f = 0; f < NF / 8; ++f) x[(k + f) % 8] = fmaf(x[(k + f) % 8], 0.999f, 1e-3f);
    }
  float t = 0.f;
  for (int k = 0; k < 8; ++k) t += c[k][0] + c[k][1] + c[k][2] + c[k][3] + x[k];
  out[blockIdx.x * blockDim.x + threadIdx.x] = t;
}

// D[block][row][col] of one 16-block 4x4x1 instruction, A = 1 + lane, B = 100 + lane
__global__ void layout_kernel(float* out) {
  const int l = threadIdx.x;
  f4 c = {0.f, 0.f, 0.f, 0.f};
  c = __builtin_amdgcn_mfma_f32_4x4x1f32(1.f + l, 100.f + l, c, 0, 0, 0);
  for (int k = 0; k < 4; ++k) out[l * 4 + k] = c[k];
}

template <class F>
float time_ms(F launch) {
  hipEvent_t e0, e1;
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));
  launch();  // warm-up
  CK(hipGetLastError());
  CK(hipEventRecord(e0));
  for (int r = 0; r < 5; ++r) launch();
  CK(hipEventRecord(e1));
  CK(hipEventSynchronize(e1));
  float ms = 0.f;
  CK(hipEventElapsedTime(&ms, e0, e1));
  CK(hipEventDestroy(e0));
  CK(hipEventDestroy(e1));
  return ms / 5.f;
}

}  // namespace

int main() {
  // --- lane layout of the 4x4x1 16-block instruction
  float* dl;
  CK(hipMalloc(&dl, 256 * sizeof(float)));
  hipLaunchKernelGGL(layout_kernel, dim3(1), dim3(64), 0, 0, dl);
  CK(hipGetLastError());
  std::vector<float> hl(256);
  CK(hipMemcpy(hl.data(), dl, 256 * sizeof(float), hipMemcpyDeviceToHost));
  int bad = 0;
  for (int l = 0; l < 64; ++l)
    for (int k = 0; k < 4; ++k)
      if (hl[l * 4 + k] != (1.f + 4 * (l / 4) + k) * (100.f + l)) ++bad;
  printf("layout: D[block][row k][col j] in register k of lane 4 block + j: %s\n", bad ? "NO" : "yes");
  CK(hipFree(dl));

  // --- the contraction, valu against mfma
  const int blocks = 256 * 16;
  std::vector<float> hpsi(PSI_FLOATS), hw(W_FLOATS);
  unsigned s = 12345u;
  auto rnd = [&]() { s = s * 1664525u + 1013904223u; return (float(s >> 8) / 16777216.f) - 0.5f; };
  for (auto& x : hpsi) x = rnd();
  for (auto& x : hw) x = rnd();
  float *gpsi, *gw, *o1, *o2;
  const size_t nout = size_t(blocks) * THREADS * 24;
  CK(hipMalloc(&gpsi, PSI_FLOATS * sizeof(float)));
  CK(hipMalloc(&gw, W_FLOATS * sizeof(float)));
  CK(hipMalloc(&o1, nout * sizeof(float)));
  CK(hipMalloc(&o2, nout * sizeof(float)));
  CK(hipMemcpy(gpsi, hpsi.data(), PSI_FLOATS * sizeof(float), hipMemcpyHostToDevice));
  CK(hipMemcpy(gw, hw.data(), W_FLOATS * sizeof(float), hipMemcpyHostToDevice));
  const float tv = time_ms([&] { hipLaunchKernelGGL(valu_kernel, dim3(blocks), dim3(THREADS), 0, 0, gpsi, gw, o1, NDIR); });
  const float tm = time_ms([&] { hipLaunchKernelGGL(mfma_kernel, dim3(blocks), dim3(THREADS), 0, 0, gpsi, gw, o2, NDIR); });
  std::vector<float> h1(size_t(THREADS) * 24), h2(size_t(THREADS) * 24);
  CK(hipMemcpy(h1.data(), o1, h1.size() * sizeof(float), hipMemcpyDeviceToHost));
  CK(hipMemcpy(h2.data(), o2, h2.size() * sizeof(float), hipMemcpyDeviceToHost));
  double num = 0, den = 0;
  for (size_t k = 0; k < h1.size(); ++k) {
    num += double(h1[k] - h2[k]) * (h1[k] - h2[k]);
    den += double(h1[k]) * h1[k];
  }
  const double lane_hops = double(blocks) * THREADS * NDIR, useful = lane_hops * 36 * 8;
  printf("contraction valu : %8.3f ms  %6.1f Tflop/s (36 complex multiply-adds per lane and hop)\n", tv,
         useful / tv / 1e9);
  printf("contraction mfma : %8.3f ms  %6.1f Tflop/s  rel-L2 vs valu %.1e\n", tm, useful / tm / 1e9,
         sqrt(num / den));
  printf("mfma / valu time : %.2f\n", tm / tv);

  // --- raw rates and overlap
  const int rb = 256 * 8, iters = 4096;
  float* dr;
  CK(hipMalloc(&dr, size_t(rb) * 256 * sizeof(float)));
  const double waves = rb * 4.0;
  const float t_m = time_ms([&] { hipLaunchKernelGGL(rate_mfma, dim3(rb), dim3(256), 0, 0, dr, iters, 1e-3f); });
  const float t_v16 = time_ms([&] { hipLaunchKernelGGL(rate_valu<16>, dim3(rb), dim3(256), 0, 0, dr, iters, 1e-3f); });
  const float t_v32 = time_ms([&] { hipLaunchKernelGGL(rate_valu<32>, dim3(rb), dim3(256), 0, 0, dr, iters, 1e-3f); });
  const float t_b16 = time_ms([&] { hipLaunchKernelGGL(rate_both<16>, dim3(rb), dim3(256), 0, 0, dr, iters, 1e-3f); });
  const float t_b32 = time_ms([&] { hipLaunchKernelGGL(rate_both<32>, dim3(rb), dim3(256), 0, 0, dr, iters, 1e-3f); });
  printf("rate mfma 4x4x1 (8/iter)         : %8.3f ms  %6.1f Tflop/s\n", t_m, waves * iters * 8 * 512 / t_m / 1e9);
  printf("rate valu fma (16/iter)          : %8.3f ms  %6.1f Tflop/s\n", t_v16, waves * iters * 16 * 128 / t_v16 / 1e9);
  printf("rate valu fma (32/iter)          : %8.3f ms  %6.1f Tflop/s\n", t_v32, waves * iters * 32 * 128 / t_v32 / 1e9);
  printf("one stream 8 mfma + 16 fma       : %8.3f ms  (sum of the parts %.3f ms)\n", t_b16, t_m + t_v16);
  printf("one stream 8 mfma + 32 fma       : %8.3f ms  (sum of the parts %.3f ms)\n", t_b32, t_m + t_v32);
  CK(hipFree(dr));
  CK(hipFree(gpsi));
  CK(hipFree(gw));
  CK(hipFree(o1));
  CK(hipFree(o2));
  return 0;
}
