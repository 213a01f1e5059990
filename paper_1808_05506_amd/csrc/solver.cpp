// Mixed-precision solve of D x = b (the paper has no solver; this is the
// defect-correction scheme of the library's C ABI).
//
//   outer (FP64):  r = b - D x;  relres_v = ||r_v|| / ||b_v||;  stop when all <= tol
//                  rhat = r / rms(r)  (per column, so 16-bit storage sees O(1) values)
//   inner (storage inner_dtype, FP32 arithmetic): CG on D^dag D e = D^dag rhat,
//                  e0 = 0, per-column alpha/beta, each column frozen once
//                  ||r_inner|| / ||r_inner,0|| <= inner_tol
//   update (FP64): x += rms(r) * e
//
// Even-odd variant (WILSON): the inner solve works on the even-site Schur
// complement M = A - H_eo A^-1 H_oe of D_W = [[A, H_eo], [H_oe, A]] in the
// packed checkerboard layout: CG on M^dag M e_e = M^dag (rhat_e - H_eo rhat_o / A),
// then e_o = (rhat_o - H_oe e_e) / A; the outer loop is unchanged.
//
// Every vector operation runs in a HIP kernel; the host only sequences the
// launches and reads the per-column norms (Nv doubles) to decide convergence.
#include "solver.hpp"

#include <math.h>
#include <stdint.h>
#include <stdio.h>

#include <vector>

#include "../../include/dslash.h"
#include "launch.hpp"

namespace dsl {

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Rows of per-workgroup partial sums the workspace holds: the reductions of
// the BLAS-1 kernels (kReduceBlocks) and of the fused D_W epilogues (one per
// workgroup; their row-staged kernels cover at least 8 sites per workgroup,
// and a launch with more workgroups falls back to the unfused form).
uint32_t partial_blocks(size_t vol) {
  const size_t b = vol / 8;
  return uint32_t(b > size_t(kReduceBlocks) ? b : size_t(kReduceBlocks));
}

struct Layout {
  size_t u_lo, e, r, p, q, s, t64, r64, partial, fold, scal, total;
  size_t field_lo, field64, links_lo;
  // even-odd only: full-lattice links before packing, the scaled residual
  // (full), its packed halves, the odd temporary and the odd solution
  size_t u_full, rfull, re, ro, tmp, eodd;
};

Layout layout_eo(const int dims[4], int nv, int lodt) {
  const size_t vol = size_t(dims[0]) * dims[1] * dims[2] * dims[3];
  Layout L;
  L.links_lo = vol * 4 * 9;
  L.field_lo = vol * 12 * nv;
  L.field64 = L.field_lo;
  const size_t half = L.field_lo / 2;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align_up(bytes);
    return o;
  };
  const size_t eb = dtype_bytes(lodt);
  L.u_lo = take(L.links_lo * eb);  // even half, then odd half
  L.u_full = take(L.links_lo * eb);
  L.rfull = take(L.field_lo * eb);
  L.re = take(half * eb);
  L.ro = take(half * eb);
  L.e = take(half * eb);
  L.r = take(half * eb);
  L.p = take(half * eb);
  L.q = take(half * eb);
  L.s = take(half * eb);
  L.tmp = take(half * eb);
  L.eodd = take(half * eb);
  L.t64 = take(L.field64 * 16);
  L.r64 = take(L.field64 * 16);
  L.partial = take(size_t(partial_blocks(vol)) * nv * sizeof(double));
  L.fold = take(size_t(kReduceBlocks) * nv * sizeof(double));
  L.scal = take(size_t(12) * nv * sizeof(double));
  L.total = off;
  return L;
}

Layout layout(int op, const int dims[4], int nv, int lodt, bool own_links) {
  const size_t vol = size_t(dims[0]) * dims[1] * dims[2] * dims[3];
  const size_t comps = size_t(spinor_comps(op));
  Layout L;
  L.links_lo = vol * links_per_site(op) * 9;
  L.field_lo = vol * comps * nv;
  L.field64 = L.field_lo;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align_up(bytes);
    return o;
  };
  const size_t eb = dtype_bytes(lodt);
  L.u_lo = own_links ? take(L.links_lo * eb) : 0;
  L.e = take(L.field_lo * eb);
  L.r = take(L.field_lo * eb);
  L.p = take(L.field_lo * eb);
  L.q = take(L.field_lo * eb);
  L.s = take(L.field_lo * eb);
  L.t64 = take(L.field64 * 16);
  L.r64 = take(L.field64 * 16);
  L.partial = take(size_t(partial_blocks(vol)) * nv * sizeof(double));
  L.fold = take(size_t(kReduceBlocks) * nv * sizeof(double));
  L.scal = take(size_t(12) * nv * sizeof(double));
  L.total = off;
  return L;
}

int hipfail(hipError_t e, const char* where) {
  char buf[256];
  snprintf(buf, sizeof buf, "%s: %s", where, hipGetErrorString(e));
  return set_error(DSLASH_E_HIP, buf);
}

#define DSL_TRY(expr, where)                         \
  do {                                               \
    hipError_t _e = (expr);                          \
    if (_e != hipSuccess) return hipfail(_e, where); \
  } while (0)

}  // namespace

size_t solve_workspace_bytes(int op, const int dims[4], int nv, int inner_dtype, bool eo, bool own_links) {
  return eo ? layout_eo(dims, nv, inner_dtype).total : layout(op, dims, nv, inner_dtype, own_links).total;
}

namespace {
// Host-side per-column values of a solve: |b|^2, |r|^2, the active flags, the
// scales, the relative residuals and the iteration counts.  Either views of the
// caller's arrays (SolveArgs::host_d / host_i: kHostDoubles / kHostInts per
// column), so that the solve allocates no memory at all, or owned vectors.
struct HostBufs {
  std::vector<double> own_d;
  std::vector<int> own_i;
  double *hb, *hr, *hact, *hsc, *relres;
  int *inner, *outer;
  int nv;
  HostBufs(int n, double* ext_d, int* ext_i) : nv(n) {
    if (!ext_d) {
      own_d.assign(size_t(kHostDoubles) * n, 0.0);
      ext_d = own_d.data();
    }
    if (!ext_i) {
      own_i.assign(size_t(kHostInts) * n, 0);
      ext_i = own_i.data();
    }
    hb = ext_d;
    hr = hb + n;
    hact = hr + n;
    hsc = hact + n;  // 2 n: scale, then its inverse
    relres = hsc + 2 * n;
    inner = ext_i;
    outer = ext_i + n;
    for (int v = 0; v < n; ++v) relres[v] = 0.0, inner[v] = 0, outer[v] = 0;
  }
  void store(const SolveArgs& a) const {
    if (a.final_relres)
      for (int v = 0; v < nv; ++v) a.final_relres[v] = relres[v];
    if (a.iters)
      for (int v = 0; v < nv; ++v) a.iters[v] = inner[v], a.iters[nv + v] = outer[v];
  }
};
}  // namespace

static int solve_eo(const SolveArgs& a);

int solve(const SolveArgs& a) {
  if (a.eo) return solve_eo(a);
  const int nv = a.nv;
  const int lodt = a.inner_dtype;
  const bool own_links = a.U_lo == nullptr;
  const Layout L = layout(a.op, a.dims, nv, lodt, own_links);
  unsigned char* ws = static_cast<unsigned char*>(a.workspace);
  const void* u_lo = own_links ? static_cast<const void*>(ws + L.u_lo) : a.U_lo;
  void* e = ws + L.e;
  void* r = ws + L.r;
  void* p = ws + L.p;
  void* q = ws + L.q;
  void* s = ws + L.s;
  void* t64 = ws + L.t64;
  void* r64 = ws + L.r64;
  double* partial = reinterpret_cast<double*>(ws + L.partial);
  double* fold = reinterpret_cast<double*>(ws + L.fold);
  double* sc = reinterpret_cast<double*>(ws + L.scal);
  double *rr = sc, *rr_new = sc + nv, *pq = sc + 2 * nv, *rr0 = sc + 3 * nv, *alpha = sc + 4 * nv,
         *beta = sc + 5 * nv, *active = sc + 6 * nv, *nb2 = sc + 7 * nv, *nr2 = sc + 8 * nv,
         *scale = sc + 9 * nv, *inv = sc + 10 * nv;
  hipStream_t st = a.stream;
  const Geom g = make_geom(a.dims, nv);
  const size_t vol = g.vol;
  const int comps = spinor_comps(a.op);
  const double nelem = double(vol) * comps;

  if (own_links)
    DSL_TRY(launch_convert(a.U64, DT_C128, ws + L.u_lo, lodt, L.links_lo, st), "link conversion");
  DSL_TRY(launch_norm2(DT_C128, a.b64, vol, comps, nv, partial, nb2, st), "norm of b");
  HostBufs h(nv, a.host_d, a.host_i);
  double *hb = h.hb, *hr = h.hr, *hact = h.hact, *hsc = h.hsc, *relres = h.relres;
  DSL_TRY(hipMemcpyAsync(hb, nb2, nv * sizeof(double), hipMemcpyDeviceToHost, st), "copy |b|^2");
  DSL_TRY(hipStreamSynchronize(st), "sync");

  int outer = 0, status = DSLASH_OK;
  for (;;) {
    // r = b - D x in FP64
    DSL_TRY(launch_apply(a.op, false, DT_C128, g, a.U64, a.x64, t64, a.mass, st), "outer apply");
    DSL_TRY(launch_xmy(a.b64, t64, r64, L.field64, st), "outer residual");
    DSL_TRY(launch_norm2(DT_C128, r64, vol, comps, nv, partial, nr2, st), "outer norm");
    DSL_TRY(hipMemcpyAsync(hr, nr2, nv * sizeof(double), hipMemcpyDeviceToHost, st), "copy |r|^2");
    DSL_TRY(hipStreamSynchronize(st), "sync");
    bool done = true;
    for (int v = 0; v < nv; ++v) {
      relres[v] = hb[v] > 0 ? sqrt(hr[v] / hb[v]) : sqrt(hr[v]);
      if (relres[v] > a.tol) done = false;
    }
    if (done) break;
    if (outer == a.max_outer) {
      status = set_error(DSLASH_E_NOCONV, "outer iteration limit reached");
      break;
    }
    ++outer;
    // per-column RMS scaling of the residual; converged columns get rhs 0 and stay frozen
    for (int v = 0; v < nv; ++v) {
      const bool work = relres[v] > a.tol && hr[v] > 0;
      const double rms = sqrt(hr[v] / nelem);
      hsc[v] = work ? rms : 0.0;
      h.outer[v] += work;
      hsc[nv + v] = work ? 1.0 / rms : 0.0;
    }
    DSL_TRY(hipMemcpyAsync(scale, hsc, 2 * nv * sizeof(double), hipMemcpyHostToDevice, st), "copy scales");
    DSL_TRY(launch_scale_to(r64, lodt, q, inv, vol, comps, nv, st), "scale residual");
    // inner CG on D^dag D e = D^dag rhat
    DSL_TRY(launch_apply(a.op, true, lodt, g, u_lo, q, r, a.mass, st), "inner rhs");
    DSL_TRY(launch_zero(lodt, e, L.field_lo, st), "zero e");
    DSL_TRY(launch_convert(r, lodt, p, lodt, L.field_lo, st), "p = r");
    DSL_TRY(launch_norm2(lodt, r, vol, comps, nv, partial, rr, st), "inner norm");
    DSL_TRY(hipMemcpyAsync(rr0, rr, nv * sizeof(double), hipMemcpyDeviceToDevice, st), "rr0");
    for (int v = 0; v < nv; ++v) hact[v] = hsc[nv + v] != 0.0 ? 1.0 : 0.0;
    DSL_TRY(hipMemcpyAsync(active, hact, nv * sizeof(double), hipMemcpyHostToDevice, st), "active");
    // One CG iteration on D^dag D: q = D p with |q|^2 fused into the apply,
    // r -= alpha D^dag q with |r|^2 fused into the adjoint apply (s never
    // stored), then e += alpha p and p = r + beta p in one pass.  Kernels
    // without the fused forms fall back to separate passes.
    for (int k = 0; k < a.max_inner; ++k) {
      EpiArgs ea;
      ea.alpha = alpha;
      ea.partial = partial;
      ea.capacity = partial_blocks(vol);
      const bool fuse = a.op == OP_WILSON && knobs().cg_fuse.get(1) != 0;
      hipError_t fe = fuse ? launch_wilson_rows(false, lodt, g, u_lo, p, q, a.mass, st, nullptr, false, EPI_NORM, &ea)
                           : hipErrorNotSupported;
      if (fe == hipSuccess) {
        DSL_TRY(launch_finish_sum(partial, int(ea.blocks), nv, pq, fold, st), "|Dp|^2");
      } else if (fe == hipErrorNotSupported) {
        DSL_TRY(launch_apply(a.op, false, lodt, g, u_lo, p, q, a.mass, st), "inner D p");
        DSL_TRY(launch_norm2(lodt, q, vol, comps, nv, partial, pq, st), "|Dp|^2");
      } else {
        return hipfail(fe, "inner D p");
      }
      DSL_TRY(launch_cg_scalars(0, nv, rr, rr_new, pq, rr0, alpha, beta, active, a.inner_tol, st), "alpha");
      fe = fuse ? launch_wilson_rows(true, lodt, g, u_lo, q, r, a.mass, st, nullptr, false, EPI_AXPY, &ea)
                : hipErrorNotSupported;
      if (fe == hipSuccess) {
        DSL_TRY(launch_finish_sum(partial, int(ea.blocks), nv, rr_new, fold, st), "|r|^2");
      } else if (fe == hipErrorNotSupported) {
        DSL_TRY(launch_apply(a.op, true, lodt, g, u_lo, q, s, a.mass, st), "inner D^dag q");
        DSL_TRY(launch_cg_update_r(lodt, r, s, alpha, vol, comps, nv, partial, rr_new, st), "r update");
      } else {
        return hipfail(fe, "inner D^dag q");
      }
      DSL_TRY(launch_cg_scalars(1, nv, rr, rr_new, pq, rr0, alpha, beta, active, a.inner_tol, st), "beta");
      DSL_TRY(launch_cg_update_ep(lodt, e, p, r, alpha, beta, vol, comps, nv, st), "e and p update");
      for (int v = 0; v < nv; ++v) h.inner[v] += hact[v] != 0.0;
      DSL_TRY(hipMemcpyAsync(hact, active, nv * sizeof(double), hipMemcpyDeviceToHost, st), "copy active");
      DSL_TRY(hipStreamSynchronize(st), "sync");
      bool any = false;
      for (int v = 0; v < nv; ++v) any = any || hact[v] != 0.0;
      if (!any) break;
    }
    DSL_TRY(launch_axpy_promote(a.x64, lodt, e, scale, vol, comps, nv, st), "x update");
  }
  h.store(a);
  return status;
}

// Even-odd inner solve (see the header comment).  Schur operator on packed
// even fields: tmp = H_oe in (odd), out = A in - H_eo tmp / A, both hops with
// the adjoint flag for M^dag.
static int solve_eo(const SolveArgs& a) {
  const int nv = a.nv;
  const int lodt = a.inner_dtype;
  const Layout L = layout_eo(a.dims, nv, lodt);
  unsigned char* ws = static_cast<unsigned char*>(a.workspace);
  const size_t eb = dtype_bytes(lodt);
  void* u_even = ws + L.u_lo;
  void* u_odd = ws + L.u_lo + L.links_lo / 2 * eb;
  void* u_full = ws + L.u_full;
  void* rfull = ws + L.rfull;
  void *re = ws + L.re, *ro = ws + L.ro, *e = ws + L.e, *r = ws + L.r, *p = ws + L.p, *q = ws + L.q, *s = ws + L.s;
  void *tmp = ws + L.tmp, *eodd = ws + L.eodd;
  void* t64 = ws + L.t64;
  void* r64 = ws + L.r64;
  double* partial = reinterpret_cast<double*>(ws + L.partial);
  double* fold = reinterpret_cast<double*>(ws + L.fold);
  double* sc = reinterpret_cast<double*>(ws + L.scal);
  double *rr = sc, *rr_new = sc + nv, *pq = sc + 2 * nv, *rr0 = sc + 3 * nv, *alpha = sc + 4 * nv,
         *beta = sc + 5 * nv, *active = sc + 6 * nv, *nb2 = sc + 7 * nv, *nr2 = sc + 8 * nv,
         *scale = sc + 9 * nv, *inv = sc + 10 * nv;
  hipStream_t st = a.stream;
  const Geom g = make_geom(a.dims, nv);
  const EoGeom eg = make_eo_geom(a.dims, nv);
  const size_t vol = g.vol, hvol = eg.hvol;
  const int comps = 12;
  const double nelem = double(vol) * comps;
  const double A = 4.0 + a.mass;
  const size_t spin_site = size_t(12) * nv * eb, link_site = size_t(36) * eb;
  const size_t half = L.field_lo / 2;

  auto schur = [&](bool adj, const void* in, void* out) -> hipError_t {
    hipError_t err = launch_wilson_eo_hop(adj, lodt, eg, 1, u_odd, u_even, in, tmp, nullptr, 0.0, 1.0, st);
    if (err != hipSuccess) return err;
    return launch_wilson_eo_hop(adj, lodt, eg, 0, u_even, u_odd, tmp, out, in, A, -1.0 / A, st);
  };

  DSL_TRY(launch_convert(a.U64, DT_C128, u_full, lodt, L.links_lo, st), "link conversion");
  DSL_TRY(launch_eo_copy(true, eg, 0, u_full, u_even, link_site, st), "pack even links");
  DSL_TRY(launch_eo_copy(true, eg, 1, u_full, u_odd, link_site, st), "pack odd links");
  DSL_TRY(launch_norm2(DT_C128, a.b64, vol, comps, nv, partial, nb2, st), "norm of b");
  HostBufs h(nv, a.host_d, a.host_i);
  double *hb = h.hb, *hr = h.hr, *hact = h.hact, *hsc = h.hsc, *relres = h.relres;
  DSL_TRY(hipMemcpyAsync(hb, nb2, nv * sizeof(double), hipMemcpyDeviceToHost, st), "copy |b|^2");
  DSL_TRY(hipStreamSynchronize(st), "sync");

  int outer = 0, status = DSLASH_OK;
  for (;;) {
    DSL_TRY(launch_apply(OP_WILSON, false, DT_C128, g, a.U64, a.x64, t64, a.mass, st), "outer apply");
    DSL_TRY(launch_xmy(a.b64, t64, r64, L.field64, st), "outer residual");
    DSL_TRY(launch_norm2(DT_C128, r64, vol, comps, nv, partial, nr2, st), "outer norm");
    DSL_TRY(hipMemcpyAsync(hr, nr2, nv * sizeof(double), hipMemcpyDeviceToHost, st), "copy |r|^2");
    DSL_TRY(hipStreamSynchronize(st), "sync");
    bool done = true;
    for (int v = 0; v < nv; ++v) {
      relres[v] = hb[v] > 0 ? sqrt(hr[v] / hb[v]) : sqrt(hr[v]);
      if (relres[v] > a.tol) done = false;
    }
    if (done) break;
    if (outer == a.max_outer) {
      status = set_error(DSLASH_E_NOCONV, "outer iteration limit reached");
      break;
    }
    ++outer;
    for (int v = 0; v < nv; ++v) {
      const bool work = relres[v] > a.tol && hr[v] > 0;
      const double rms = sqrt(hr[v] / nelem);
      hsc[v] = work ? rms : 0.0;
      h.outer[v] += work;
      hsc[nv + v] = work ? 1.0 / rms : 0.0;
    }
    DSL_TRY(hipMemcpyAsync(scale, hsc, 2 * nv * sizeof(double), hipMemcpyHostToDevice, st), "copy scales");
    DSL_TRY(launch_scale_to(r64, lodt, rfull, inv, vol, comps, nv, st), "scale residual");
    DSL_TRY(launch_eo_copy(true, eg, 0, rfull, re, spin_site, st), "pack even residual");
    DSL_TRY(launch_eo_copy(true, eg, 1, rfull, ro, spin_site, st), "pack odd residual");
    // Schur right-hand side rhat_e - H_eo rhat_o / A, then CG on M^dag M
    DSL_TRY(launch_wilson_eo_hop(false, lodt, eg, 0, u_even, u_odd, ro, q, re, 1.0, -1.0 / A, st), "Schur rhs");
    DSL_TRY(schur(true, q, r), "inner rhs");
    DSL_TRY(launch_zero(lodt, e, half, st), "zero e");
    DSL_TRY(launch_convert(r, lodt, p, lodt, half, st), "p = r");
    DSL_TRY(launch_norm2(lodt, r, hvol, comps, nv, partial, rr, st), "inner norm");
    DSL_TRY(hipMemcpyAsync(rr0, rr, nv * sizeof(double), hipMemcpyDeviceToDevice, st), "rr0");
    for (int v = 0; v < nv; ++v) hact[v] = hsc[nv + v] != 0.0 ? 1.0 : 0.0;
    DSL_TRY(hipMemcpyAsync(active, hact, nv * sizeof(double), hipMemcpyHostToDevice, st), "active");
    // CG on M^dag M with the same fusions as the full-lattice loop: |q|^2 in
    // the second hop of q = M p, r -= alpha M^dag q in the second hop of M^dag q
    for (int k = 0; k < a.max_inner; ++k) {
      EpiArgs ea;
      ea.alpha = alpha;
      ea.partial = partial;
      ea.capacity = partial_blocks(vol);
      const bool fuse = knobs().cg_fuse.get(1) != 0;
      DSL_TRY(launch_wilson_eo_hop(false, lodt, eg, 1, u_odd, u_even, p, tmp, nullptr, 0.0, 1.0, st), "inner M p");
      hipError_t fe = fuse ? launch_wilson_eo_hop(false, lodt, eg, 0, u_even, u_odd, tmp, q, p, A, -1.0 / A, st,
                                                  EPI_NORM, &ea)
                           : hipErrorNotSupported;
      if (fe == hipSuccess) {
        DSL_TRY(launch_finish_sum(partial, int(ea.blocks), nv, pq, fold, st), "|Mp|^2");
      } else if (fe == hipErrorNotSupported) {
        DSL_TRY(launch_wilson_eo_hop(false, lodt, eg, 0, u_even, u_odd, tmp, q, p, A, -1.0 / A, st), "inner M p");
        DSL_TRY(launch_norm2(lodt, q, hvol, comps, nv, partial, pq, st), "|Mp|^2");
      } else {
        return hipfail(fe, "inner M p");
      }
      DSL_TRY(launch_cg_scalars(0, nv, rr, rr_new, pq, rr0, alpha, beta, active, a.inner_tol, st), "alpha");
      DSL_TRY(launch_wilson_eo_hop(true, lodt, eg, 1, u_odd, u_even, q, tmp, nullptr, 0.0, 1.0, st), "inner M^dag q");
      fe = fuse ? launch_wilson_eo_hop(true, lodt, eg, 0, u_even, u_odd, tmp, r, q, A, -1.0 / A, st, EPI_AXPY, &ea)
                : hipErrorNotSupported;
      if (fe == hipSuccess) {
        DSL_TRY(launch_finish_sum(partial, int(ea.blocks), nv, rr_new, fold, st), "|r|^2");
      } else if (fe == hipErrorNotSupported) {
        DSL_TRY(launch_wilson_eo_hop(true, lodt, eg, 0, u_even, u_odd, tmp, s, q, A, -1.0 / A, st), "inner M^dag q");
        DSL_TRY(launch_cg_update_r(lodt, r, s, alpha, hvol, comps, nv, partial, rr_new, st), "r update");
      } else {
        return hipfail(fe, "inner M^dag q");
      }
      DSL_TRY(launch_cg_scalars(1, nv, rr, rr_new, pq, rr0, alpha, beta, active, a.inner_tol, st), "beta");
      DSL_TRY(launch_cg_update_ep(lodt, e, p, r, alpha, beta, hvol, comps, nv, st), "e and p update");
      for (int v = 0; v < nv; ++v) h.inner[v] += hact[v] != 0.0;
      DSL_TRY(hipMemcpyAsync(hact, active, nv * sizeof(double), hipMemcpyDeviceToHost, st), "copy active");
      DSL_TRY(hipStreamSynchronize(st), "sync");
      bool any = false;
      for (int v = 0; v < nv; ++v) any = any || hact[v] != 0.0;
      if (!any) break;
    }
    // odd half e_o = (rhat_o - H_oe e_e) / A, then the full correction
    DSL_TRY(launch_wilson_eo_hop(false, lodt, eg, 1, u_odd, u_even, e, eodd, ro, 1.0 / A, -1.0 / A, st), "odd half");
    DSL_TRY(launch_eo_copy(false, eg, 0, e, rfull, spin_site, st), "unpack even");
    DSL_TRY(launch_eo_copy(false, eg, 1, eodd, rfull, spin_site, st), "unpack odd");
    DSL_TRY(launch_axpy_promote(a.x64, lodt, rfull, scale, vol, comps, nv, st), "x update");
  }
  h.store(a);
  return status;
}

}  // namespace dsl
