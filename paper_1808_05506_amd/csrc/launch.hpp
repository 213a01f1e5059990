// Internal launcher interface between the C ABI / solver (host C++) and the
// HIP kernels.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>

#include "dslash_common.hpp"

namespace dsl {

// Tuning knobs: the environment variables DSLASH_<NAME>, read once per process
// (at the first launch that consults them) and again only on an explicit
// reload (dslash_reload_tuning), so the kernel choice does not change during a
// run and launches pay no lookups.  A knob that is not set leaves the
// launcher's default.
struct Knob {
  bool set = false;
  int value = 0;
  int get(int dflt) const { return set ? value : dflt; }
};
struct Knobs {
  Knob sites_per_block, tband, xcd, row_sites, row_depth, tsteps, march_pp, rows, row_lds_extra, cg_fuse;
  Knob grad_tile_y, grad_tile_z, march_tile_y, march_tile_z, bri_tile_y, bri_tile_z, rows_tile_y,
      rows_tile_z, blas_nt, wmarch_tile_y, wmarch_tile_z;
};
inline Knob read_knob(const char* name) {
  Knob k;
  if (const char* e = getenv(name)) {
    k.set = true;
    k.value = atoi(e);
  }
  return k;
}
inline Knobs read_knobs() {
  Knobs r;
  r.sites_per_block = read_knob("DSLASH_SITES_PER_BLOCK");
  r.tband = read_knob("DSLASH_TBAND");
  r.xcd = read_knob("DSLASH_XCD");
  r.row_sites = read_knob("DSLASH_ROW_SITES");
  r.row_depth = read_knob("DSLASH_ROW_DEPTH");
  r.tsteps = read_knob("DSLASH_TSTEPS");
  r.march_pp = read_knob("DSLASH_MARCH_PP");
  r.rows = read_knob("DSLASH_ROWS");
  r.row_lds_extra = read_knob("DSLASH_ROW_LDS_EXTRA");
  r.cg_fuse = read_knob("DSLASH_CG_FUSE");
  r.grad_tile_y = read_knob("DSLASH_GRAD_TILE_Y");
  r.grad_tile_z = read_knob("DSLASH_GRAD_TILE_Z");
  r.march_tile_y = read_knob("DSLASH_MARCH_TILE_Y");
  r.march_tile_z = read_knob("DSLASH_MARCH_TILE_Z");
  r.bri_tile_y = read_knob("DSLASH_BRI_TILE_Y");
  r.bri_tile_z = read_knob("DSLASH_BRI_TILE_Z");
  r.rows_tile_y = read_knob("DSLASH_ROWS_TILE_Y");
  r.rows_tile_z = read_knob("DSLASH_ROWS_TILE_Z");
  r.blas_nt = read_knob("DSLASH_BLAS_NT");
  r.wmarch_tile_y = read_knob("DSLASH_WMARCH_TILE_Y");
  r.wmarch_tile_z = read_knob("DSLASH_WMARCH_TILE_Z");
  return r;
}
inline Knobs& knob_store() {
  static Knobs k = read_knobs();
  return k;
}
inline const Knobs& knobs() { return knob_store(); }

enum Op { OP_STAGGERED = 0, OP_WILSON = 1, OP_BRILLOUIN = 2 };
enum Dtype { DT_C64 = 0, DT_C128 = 1, DT_BF16 = 2, DT_F16 = 3 };

// Field pointers of the kernels that move 16-byte pieces must be 16-byte
// aligned (every torch allocation is); others take the per-word kernels.
inline bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

inline size_t dtype_bytes(int dt) { return dt == DT_C128 ? 16 : dt == DT_C64 ? 8 : 4; }
inline int spinor_comps(int op) { return op == OP_STAGGERED ? 3 : 12; }
inline int links_per_site(int op) { return op == OP_BRILLOUIN ? 40 : 4; }

Geom make_geom(const int dims[4], int nv);

// Thread shape of the (site, right-hand side) kernels.
struct Shape {
  dim3 grid, block;
};
Shape site_v_shape(uint32_t vol, int nv);

// clover: packed site-local clover term (36 words per site) added to D_W or
// D_B, or nullptr; STAGGERED takes none.  compressed: U holds the first two
// rows of every link (6 words per link; STAGGERED and WILSON, not with clover).
hipError_t launch_apply(int op, bool adjoint, int dtype, const Geom& g, const void* U, const void* in, void* out,
                        double mass, hipStream_t st, const void* clover = nullptr, bool compressed = false);
// epi, ea: fused output epilogue (EPI_*, EpiArgs: the solver's D with EPI_NORM
// and D^dag with EPI_AXPY on the t-marching kernels); hipErrorNotSupported
// when the chosen kernel has no such form.
hipError_t launch_wilson_rows(bool adjoint, int dtype, const Geom& g, const void* U, const void* in, void* out,
                              double mass, hipStream_t st, const void* clover = nullptr, bool compressed = false,
                              int epi = 0, EpiArgs* ea = nullptr);
hipError_t launch_staggered_rows(bool adjoint, int dtype, const Geom& g, const void* U, const void* in, void* out,
                                 double mass, hipStream_t st, bool compressed = false);
hipError_t launch_compress_links(int dtype, size_t links, const void* V, void* Vc, hipStream_t st);
hipError_t launch_brillouin_rows(bool adjoint, int dtype, const Geom& g, const void* W, const void* in, void* out,
                                 double mass, hipStream_t st, const void* clover = nullptr);
hipError_t launch_brillouin_links(int dtype, const Geom& g, const void* V, void* W, hipStream_t st);
hipError_t launch_brillouin_fly(bool adjoint, int dtype, const Geom& g, const void* V, const void* in, void* out,
                                double mass, hipStream_t st, const void* clover = nullptr);
hipError_t launch_clover_field(int dtype, const Geom& g, const void* V, void* C, double c_sw, hipStream_t st);
hipError_t launch_brillouin_wgrad(int dtype, const Geom& g, const void* chi, const void* psi, void* GW,
                                  hipStream_t st);
hipError_t launch_brillouin_wgrad_rows(int dtype, const Geom& g, const void* chi, const void* psi, void* GW,
                                       hipStream_t st);
// W (nullable): the stored off-axis links of V; with it the adjoint uses the
// path averages of W instead of walking every ordering through V
hipError_t launch_brillouin_links_backward(int dtype, const Geom& g, const void* V, const void* W, const void* GW,
                                           void* GV, hipStream_t st);
// W built level by level from the first-hop recursion of the path averages.
hipError_t launch_brillouin_links_levels(int dtype, const Geom& g, const void* V, void* W, hipStream_t st);
// The same through the level recursion of the path averages; ws: 756 words a site.
hipError_t launch_brillouin_links_backward_levels(int dtype, const Geom& g, const void* V, const void* W,
                                                  const void* GW, void* GV, void* ws, hipStream_t st);
hipError_t launch_link_grad(int op, int dtype, const Geom& g, const void* chi, const void* psi, void* G,
                            hipStream_t st);
hipError_t launch_grad_rows(int op, int dtype, const Geom& g, const void* chi, const void* psi, void* G,
                            hipStream_t st);
hipError_t launch_convert(const void* src, int sdt, void* dst, int ddt, size_t n, hipStream_t st);

// ---- even-odd (checkerboard) form of D_W (eo.hip)
struct EoGeom {
  int n[4];       // full extents (all even)
  int nh;         // Nx / 2: packed sites per row
  uint32_t hvol;  // sites of one parity
  int nv;
  FastDiv dnh, dy, dz;
};
EoGeom make_eo_geom(const int dims[4], int nv);
// full <-> packed parity `parity` copy of `site_bytes` bytes per site
hipError_t launch_eo_copy(bool to_packed, const EoGeom& e, int parity, const void* src, void* dst, size_t site_bytes,
                          hipStream_t st);
// out = c_add add + c_hop H in on the packed parity-`parity` sites (add may be null)
// epi, ea: fused output epilogue as for launch_wilson_rows (the Schur operator
// M with EPI_NORM, M^dag with EPI_AXPY; row-staged kernel only)
hipError_t launch_wilson_eo_hop(bool adj, int dtype, const EoGeom& e, int parity, const void* Uo, const void* Ui,
                                const void* in, void* out, const void* add, double c_add, double c_hop,
                                hipStream_t st, int epi = 0, EpiArgs* ea = nullptr);
hipError_t launch_wilson_eo_rows(bool adj, int dtype, const EoGeom& e, int parity, const void* Uo, const void* Ui,
                                 const void* in, void* out, const void* add, double c_add, double c_hop,
                                 hipStream_t st, int epi = 0, EpiArgs* ea = nullptr);

// ---- solver BLAS-1 (fields of `comps` complex numbers per site times nv columns,
//      column index fastest; per-column scalars are device arrays of nv doubles)
constexpr int kReduceBlocks = 512;
// partial[b][v] = sum over the block's sites of |x|^2 (FP64), then out[v] = sum_b partial[b][v]
hipError_t launch_norm2(int dtype, const void* x, size_t sites, int comps, int nv, double* partial, double* out,
                        hipStream_t st);
// r = b - t (all C128)
hipError_t launch_xmy(const void* b, const void* t, void* r, size_t n, hipStream_t st);
// lo = hi * inv[v] (hi C128 -> lo dtype)
hipError_t launch_scale_to(const void* hi, int lodt, void* lo, const double* inv, size_t sites, int comps, int nv,
                           hipStream_t st);
// x += s[v] * e  (x C128, e lo dtype)
hipError_t launch_axpy_promote(void* x, int lodt, const void* e, const double* s, size_t sites, int comps, int nv,
                               hipStream_t st);
// e += alpha[v] p;  r -= alpha[v] q;  partial |r|^2 -> out
hipError_t launch_cg_update_xr(int dtype, void* e, void* r, const void* p, const void* q, const double* alpha,
                               size_t sites, int comps, int nv, double* partial, double* out, hipStream_t st);
// r -= alpha[v] s;  partial |r|^2 -> out
hipError_t launch_cg_update_r(int dtype, void* r, const void* s, const double* alpha, size_t sites, int comps, int nv,
                              double* partial, double* out, hipStream_t st);
// e += alpha[v] p;  p = r + beta[v] p
hipError_t launch_cg_update_ep(int dtype, void* e, void* p, const void* r, const double* alpha, const double* beta,
                               size_t sites, int comps, int nv, hipStream_t st);
// out[v] = sum over b < nb of partial[b][v], in a fixed order (many rows are
// first folded to kReduceBlocks rows in fold, kReduceBlocks x nv doubles)
hipError_t launch_finish_sum(const double* partial, int nb, int nv, double* out, double* fold, hipStream_t st);
// p = r + beta[v] p
hipError_t launch_cg_update_p(int dtype, void* p, const void* r, const double* beta, size_t sites, int comps,
                              int nv, hipStream_t st);
// zero n complex numbers of dtype
hipError_t launch_zero(int dtype, void* x, size_t n, hipStream_t st);
// per-column CG scalars on the device (see solver.cpp):
//   mode 0: alpha = active ? rr / pq : 0
//   mode 1: beta = active ? rr_new / rr : 0; rr = active ? rr_new : rr;
//           active &= sqrt(rr / rr0) > tol
hipError_t launch_cg_scalars(int mode, int nv, double* rr, double* rr_new, double* pq, double* rr0, double* alpha,
                             double* beta, double* active, double tol, hipStream_t st);

}  // namespace dsl
