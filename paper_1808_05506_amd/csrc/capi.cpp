// C ABI of the Dirac-operator library (declared in include/dslash.h).
//
// Every entry point validates its arguments synchronously, before any HIP
// call, and reports failures as status codes with a thread-local detail
// string; nothing is thrown across the ABI.
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <mutex>

#include "../../include/dslash.h"
#include "launch.hpp"
#include "solver.hpp"

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}

int hip_fail(hipError_t e, const char* where) {
  return fail(DSLASH_E_HIP, "%s: %s", where, hipGetErrorString(e));
}

bool valid_dtype(int dt) { return dt >= DSLASH_C64 && dt <= DSLASH_F16; }

// Common checks on lattice geometry and sizes.
int check_geom(int op, const int dims[4], int Nc, int Nv) {
  if (!dims) return fail(DSLASH_E_ARG, "dims is NULL");
  if (op < DSLASH_STAGGERED || op > DSLASH_BRILLOUIN) return fail(DSLASH_E_ARG, "unknown op %d", op);
  if (Nc != 3) return fail(DSLASH_E_UNSUPPORTED, "only Nc = 3 is built (got %d)", Nc);
  if (Nv < 1) return fail(DSLASH_E_ARG, "Nv must be >= 1 (got %d)", Nv);
  uint64_t vol = 1;
  for (int i = 0; i < 4; ++i) {
    if (dims[i] < 2) return fail(DSLASH_E_ARG, "dims[%d] = %d < 2", i, dims[i]);
    if (op == DSLASH_STAGGERED && (dims[i] & 1))
      return fail(DSLASH_E_ARG, "staggered operator needs even extents (dims[%d] = %d)", i, dims[i]);
    vol *= uint64_t(dims[i]);
  }
  if (vol >= (1ull << 31)) return fail(DSLASH_E_ARG, "lattice volume %llu >= 2^31", (unsigned long long)vol);
  return DSLASH_OK;
}

uint64_t volume(const int dims[4]) { return uint64_t(dims[0]) * dims[1] * dims[2] * dims[3]; }

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t pa = uintptr_t(a), pb = uintptr_t(b);
  return pa < pb + nb && pb < pa + na;
}

}  // namespace

namespace dsl {
int set_error(int code, const char* msg) { return fail(code, "%s", msg); }
}  // namespace dsl

extern "C" {

const char* dslash_status_string(int status) {
  switch (status) {
    case DSLASH_OK: return "ok";
    case DSLASH_E_ARG: return "invalid argument";
    case DSLASH_E_UNSUPPORTED: return "unsupported configuration";
    case DSLASH_E_ALIAS: return "output aliases an input";
    case DSLASH_E_HIP: return "HIP runtime error";
    case DSLASH_E_NOCONV: return "solver did not converge";
    case DSLASH_E_WORKSPACE: return "workspace missing or too small";
  }
  return "unknown status";
}

const char* dslash_last_error(void) { return g_err; }

int dslash_version(void) { return 201; }

int dslash_reload_tuning(void) {
  dsl::knob_store() = dsl::read_knobs();
  return DSLASH_OK;
}

static int apply_common(bool adj, int op, const void* U, const void* in, void* out, const int dims[4], int Nc,
                        int Nv, double mass, int dtype, void* stream, const void* C = nullptr,
                        bool compressed = false) {
  g_err[0] = 0;
  if (int rc = check_geom(op, dims, Nc, Nv)) return rc;
  if (!valid_dtype(dtype)) return fail(DSLASH_E_ARG, "unknown dtype %d", dtype);
  if (!U || !in || !out) return fail(DSLASH_E_ARG, "NULL field pointer");
  const uint64_t vol = volume(dims);
  const size_t eb = dsl::dtype_bytes(dtype);
  const size_t nspin = size_t(vol) * dsl::spinor_comps(op) * Nv * eb;
  const size_t nlink = size_t(vol) * dsl::links_per_site(op) * (compressed ? 6 : 9) * eb;
  if (overlap(in, nspin, out, nspin)) return fail(DSLASH_E_ALIAS, "in and out overlap");
  if (overlap(U, nlink, out, nspin)) return fail(DSLASH_E_ALIAS, "U and out overlap");
  if (C && overlap(C, size_t(vol) * 36 * eb, out, nspin)) return fail(DSLASH_E_ALIAS, "C and out overlap");
  const dsl::Geom g = dsl::make_geom(dims, Nv);
  hipError_t e = dsl::launch_apply(op, adj, dtype, g, U, in, out, mass, (hipStream_t)stream, C, compressed);
  if (e != hipSuccess) return hip_fail(e, "dslash_apply launch");
  return DSLASH_OK;
}

int dslash_apply(int op, const void* U, const void* in, void* out, const int dims[4], int Nc, int Nv, double mass,
                 int dtype, void* stream) {
  return apply_common(false, op, U, in, out, dims, Nc, Nv, mass, dtype, stream);
}

int dslash_apply_adjoint(int op, const void* U, const void* in, void* out, const int dims[4], int Nc, int Nv,
                         double mass, int dtype, void* stream) {
  return apply_common(true, op, U, in, out, dims, Nc, Nv, mass, dtype, stream);
}

int dslash_clover_field(const void* V, void* C, const int dims[4], int Nc, double c_sw, int dtype, void* stream) {
  g_err[0] = 0;
  if (int rc = check_geom(DSLASH_WILSON, dims, Nc, 1)) return rc;
  if (!valid_dtype(dtype)) return fail(DSLASH_E_ARG, "unknown dtype %d", dtype);
  if (!V || !C) return fail(DSLASH_E_ARG, "NULL field pointer");
  const uint64_t vol = volume(dims);
  const size_t eb = dsl::dtype_bytes(dtype);
  if (overlap(V, size_t(vol) * 36 * eb, C, size_t(vol) * 36 * eb)) return fail(DSLASH_E_ALIAS, "V and C overlap");
  const dsl::Geom g = dsl::make_geom(dims, 1);
  hipError_t e = dsl::launch_clover_field(dtype, g, V, C, c_sw, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "dslash_clover_field launch");
  return DSLASH_OK;
}

int dslash_apply_clover(int op, const void* U, const void* C, const void* in, void* out, const int dims[4], int Nc,
                        int Nv, double mass, int adjoint, int dtype, void* stream) {
  g_err[0] = 0;
  if (op != DSLASH_WILSON && op != DSLASH_BRILLOUIN)
    return fail(DSLASH_E_ARG, "the clover term belongs to WILSON and BRILLOUIN (got op %d)", op);
  if (!C) return fail(DSLASH_E_ARG, "C is NULL");
  return apply_common(adjoint != 0, op, U, in, out, dims, Nc, Nv, mass, dtype, stream, C);
}

int dslash_compress_links(const void* V, void* Vc, const int dims[4], int Nc, int dtype, void* stream) {
  g_err[0] = 0;
  if (int rc = check_geom(DSLASH_WILSON, dims, Nc, 1)) return rc;
  if (!valid_dtype(dtype)) return fail(DSLASH_E_ARG, "unknown dtype %d", dtype);
  if (!V || !Vc) return fail(DSLASH_E_ARG, "NULL field pointer");
  const uint64_t vol = volume(dims);
  const size_t eb = dsl::dtype_bytes(dtype);
  if (overlap(V, size_t(vol) * 36 * eb, Vc, size_t(vol) * 24 * eb)) return fail(DSLASH_E_ALIAS, "V and Vc overlap");
  hipError_t e = dsl::launch_compress_links(dtype, size_t(vol) * 4, V, Vc, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "dslash_compress_links launch");
  return DSLASH_OK;
}

int dslash_apply_compressed(int op, const void* Vc, const void* in, void* out, const int dims[4], int Nc, int Nv,
                            double mass, int adjoint, int dtype, void* stream) {
  g_err[0] = 0;
  if (op != DSLASH_STAGGERED && op != DSLASH_WILSON)
    return fail(DSLASH_E_ARG, "compressed links are built for STAGGERED and WILSON (got op %d)", op);
  return apply_common(adjoint != 0, op, Vc, in, out, dims, Nc, Nv, mass, dtype, stream, nullptr, true);
}

int dslash_apply_brillouin_fly(const void* V, const void* in, void* out, const int dims[4], int Nc, int Nv,
                               double mass, int adjoint, int dtype, void* stream) {
  g_err[0] = 0;
  if (int rc = check_geom(DSLASH_BRILLOUIN, dims, Nc, Nv)) return rc;
  if (!valid_dtype(dtype)) return fail(DSLASH_E_ARG, "unknown dtype %d", dtype);
  if (!V || !in || !out) return fail(DSLASH_E_ARG, "NULL field pointer");
  const uint64_t vol = volume(dims);
  const size_t eb = dsl::dtype_bytes(dtype);
  const size_t nspin = size_t(vol) * 12 * Nv * eb, nlink = size_t(vol) * 36 * eb;
  if (overlap(in, nspin, out, nspin)) return fail(DSLASH_E_ALIAS, "in and out overlap");
  if (overlap(V, nlink, out, nspin)) return fail(DSLASH_E_ALIAS, "V and out overlap");
  const dsl::Geom g = dsl::make_geom(dims, Nv);
  hipError_t e = dsl::launch_brillouin_fly(adjoint != 0, dtype, g, V, in, out, mass, (hipStream_t)stream);
  if (e == hipErrorNotSupported)
    return fail(DSLASH_E_UNSUPPORTED,
                "on-the-fly links are built for N_v = 4, 8, 12, 16, 24, C64 and the rows the row-staged kernel "
                "covers (got N_v = %d, dtype %d, Nx = %d)", Nv, dtype, dims[0]);
  if (e != hipSuccess) return hip_fail(e, "dslash_apply_brillouin_fly launch");
  return DSLASH_OK;
}

int dslash_backward(int op, const void* U, const void* grad_out, const void* in, void* grad_U, void* grad_in,
                    const int dims[4], int Nc, int Nv, double mass, int dtype, void* stream) {
  g_err[0] = 0;
  if (int rc = check_geom(op, dims, Nc, Nv)) return rc;
  if (dtype != DSLASH_C64 && dtype != DSLASH_C128)
    return fail(DSLASH_E_UNSUPPORTED, "backward is built for C64 and C128 only (got dtype %d)", dtype);
  if (!grad_out) return fail(DSLASH_E_ARG, "grad_out is NULL");
  if (grad_in && !U) return fail(DSLASH_E_ARG, "U is NULL but grad_in requested");
  if (grad_U && !in) return fail(DSLASH_E_ARG, "in is NULL but grad_U requested");
  const uint64_t vol = volume(dims);
  const size_t eb = dsl::dtype_bytes(dtype);
  const size_t nspin = size_t(vol) * dsl::spinor_comps(op) * Nv * eb;
  const size_t nlink = size_t(vol) * dsl::links_per_site(op) * 9 * eb;
  if (grad_in) {
    if (overlap(grad_in, nspin, grad_out, nspin) || (in && overlap(grad_in, nspin, in, nspin)) ||
        overlap(grad_in, nspin, U, nlink))
      return fail(DSLASH_E_ALIAS, "grad_in overlaps an input");
  }
  if (grad_U) {
    if (overlap(grad_U, nlink, grad_out, nspin) || overlap(grad_U, nlink, in, nspin) ||
        (U && overlap(grad_U, nlink, U, nlink)) || (grad_in && overlap(grad_U, nlink, grad_in, nspin)))
      return fail(DSLASH_E_ALIAS, "grad_U overlaps another argument");
  }
  const dsl::Geom g = dsl::make_geom(dims, Nv);
  hipStream_t st = (hipStream_t)stream;
  if (grad_in) {
    hipError_t e = dsl::launch_apply(op, true, dtype, g, U, grad_out, grad_in, mass, st);
    if (e != hipSuccess) return hip_fail(e, "dslash_backward grad_in launch");
  }
  if (grad_U) {
    hipError_t e = op == DSLASH_BRILLOUIN ? dsl::launch_brillouin_wgrad(dtype, g, grad_out, in, grad_U, st)
                                          : dsl::launch_link_grad(op, dtype, g, grad_out, in, grad_U, st);
    if (e != hipSuccess) return hip_fail(e, "dslash_backward grad_U launch");
  }
  return DSLASH_OK;
}

int dslash_brillouin_links_backward(const void* V, const void* W, const void* grad_W, void* grad_V, const int dims[4],
                                    int Nc, int dtype, void* stream) {
  g_err[0] = 0;
  if (int rc = check_geom(DSLASH_BRILLOUIN, dims, Nc, 1)) return rc;
  if (dtype != DSLASH_C64 && dtype != DSLASH_C128)
    return fail(DSLASH_E_UNSUPPORTED, "W construction is built for C64 and C128 only (got dtype %d)", dtype);
  if (!V || !grad_W || !grad_V) return fail(DSLASH_E_ARG, "NULL field pointer");
  const uint64_t vol = volume(dims);
  const size_t eb = dsl::dtype_bytes(dtype);
  const size_t nv = size_t(vol) * 36 * eb, nw = size_t(vol) * 360 * eb;
  if (overlap(grad_V, nv, V, nv) || overlap(grad_V, nv, grad_W, nw) || (W && overlap(grad_V, nv, W, nw)))
    return fail(DSLASH_E_ALIAS, "grad_V overlaps an input");
  const dsl::Geom g = dsl::make_geom(dims, 1);
  hipError_t e = dsl::launch_brillouin_links_backward(dtype, g, V, W, grad_W, grad_V, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "dslash_brillouin_links_backward launch");
  return DSLASH_OK;
}

size_t dslash_brillouin_links_backward_workspace_bytes(const int dims[4], int Nc, int dtype) {
  if (check_geom(DSLASH_BRILLOUIN, dims, Nc, 1)) return 0;
  if (dtype != DSLASH_C64 && dtype != DSLASH_C128) return 0;
  return size_t(volume(dims)) * 756 * dsl::dtype_bytes(dtype);
}

int dslash_brillouin_links_backward_ws(const void* V, const void* W, const void* grad_W, void* grad_V, void* workspace,
                                       size_t ws_bytes, const int dims[4], int Nc, int dtype, void* stream) {
  g_err[0] = 0;
  if (int rc = check_geom(DSLASH_BRILLOUIN, dims, Nc, 1)) return rc;
  if (dtype != DSLASH_C64 && dtype != DSLASH_C128)
    return fail(DSLASH_E_UNSUPPORTED, "W construction is built for C64 and C128 only (got dtype %d)", dtype);
  if (!V || !W || !grad_W || !grad_V) return fail(DSLASH_E_ARG, "NULL field pointer");
  if (!workspace) return fail(DSLASH_E_ARG, "NULL workspace");
  if (reinterpret_cast<uintptr_t>(workspace) % 16 != 0) return fail(DSLASH_E_ARG, "workspace not 16-byte aligned");
  const uint64_t vol = volume(dims);
  const size_t eb = dsl::dtype_bytes(dtype);
  const size_t nv = size_t(vol) * 36 * eb, nw = size_t(vol) * 360 * eb;
  const size_t nws = size_t(vol) * 756 * eb;
  if (ws_bytes < nws) return fail(DSLASH_E_ARG, "workspace of %zu bytes, %zu needed", ws_bytes, nws);
  if (overlap(grad_V, nv, V, nv) || overlap(grad_V, nv, grad_W, nw) || overlap(grad_V, nv, W, nw))
    return fail(DSLASH_E_ALIAS, "grad_V overlaps an input");
  if (overlap(workspace, nws, V, nv) || overlap(workspace, nws, W, nw) || overlap(workspace, nws, grad_W, nw) ||
      overlap(workspace, nws, grad_V, nv))
    return fail(DSLASH_E_ALIAS, "workspace overlaps another argument");
  const dsl::Geom g = dsl::make_geom(dims, 1);
  hipError_t e =
      dsl::launch_brillouin_links_backward_levels(dtype, g, V, W, grad_W, grad_V, workspace, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "dslash_brillouin_links_backward_ws launch");
  return DSLASH_OK;
}

int dslash_brillouin_links(const void* V, void* W, const int dims[4], int Nc, int dtype, void* stream) {
  g_err[0] = 0;
  if (int rc = check_geom(DSLASH_BRILLOUIN, dims, Nc, 1)) return rc;
  if (dtype != DSLASH_C64 && dtype != DSLASH_C128)
    return fail(DSLASH_E_UNSUPPORTED, "W construction is built for C64 and C128 only (got dtype %d)", dtype);
  if (!V || !W) return fail(DSLASH_E_ARG, "NULL field pointer");
  const uint64_t vol = volume(dims);
  const size_t eb = dsl::dtype_bytes(dtype);
  if (overlap(V, size_t(vol) * 36 * eb, W, size_t(vol) * 360 * eb)) return fail(DSLASH_E_ALIAS, "V and W overlap");
  const dsl::Geom g = dsl::make_geom(dims, 1);
  hipError_t e = dsl::launch_brillouin_links(dtype, g, V, W, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "dslash_brillouin_links launch");
  return DSLASH_OK;
}

int dslash_convert(const void* src, int src_dtype, void* dst, int dst_dtype, size_t n, void* stream) {
  g_err[0] = 0;
  if (!valid_dtype(src_dtype) || !valid_dtype(dst_dtype)) return fail(DSLASH_E_ARG, "unknown dtype");
  if (n == 0) return DSLASH_OK;
  if (!src || !dst) return fail(DSLASH_E_ARG, "NULL pointer");
  if (overlap(src, n * dsl::dtype_bytes(src_dtype), dst, n * dsl::dtype_bytes(dst_dtype)))
    return fail(DSLASH_E_ALIAS, "src and dst overlap");
  hipError_t e = dsl::launch_convert(src, src_dtype, dst, dst_dtype, n, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "dslash_convert launch");
  return DSLASH_OK;
}

static bool valid_inner(int dt) { return dt == DSLASH_C64 || dt == DSLASH_BF16 || dt == DSLASH_F16; }

// Checks shared by the solve entry points; fills a with everything but the
// workspace, the caller's links and the eo flag.
static int solve_args(int op, const void* U64, const void* b64, void* x64, const int dims[4], int Nc, int Nv,
                      double mass, int inner_dtype, double tol, double inner_tol, int max_outer, int max_inner,
                      double* final_relres, int* iters, void* stream, dsl::SolveArgs& a) {
  if (int rc = check_geom(op, dims, Nc, Nv)) return rc;
  if (op == DSLASH_BRILLOUIN) return fail(DSLASH_E_ARG, "the solver is built for STAGGERED and WILSON (got BRILLOUIN)");
  if (!valid_inner(inner_dtype))
    return fail(DSLASH_E_ARG, "inner dtype must be C64, BF16 or F16 (got %d)", inner_dtype);
  if (!U64 || !b64 || !x64) return fail(DSLASH_E_ARG, "NULL field pointer");
  if (!(tol > 0) || !(inner_tol > 0) || !(inner_tol < 1)) return fail(DSLASH_E_ARG, "need tol > 0, 0 < inner_tol < 1");
  if (max_outer < 1 || max_inner < 1) return fail(DSLASH_E_ARG, "iteration limits must be >= 1");
  const uint64_t vol = volume(dims);
  const size_t nspin = size_t(vol) * dsl::spinor_comps(op) * Nv * 16;
  const size_t nlink = size_t(vol) * dsl::links_per_site(op) * 9 * 16;
  if (overlap(x64, nspin, b64, nspin) || overlap(x64, nspin, U64, nlink))
    return fail(DSLASH_E_ALIAS, "x must not overlap b or U");
  a.op = op;
  a.U64 = U64;
  a.b64 = b64;
  a.x64 = x64;
  for (int i = 0; i < 4; ++i) a.dims[i] = dims[i];
  a.nv = Nv;
  a.mass = mass;
  a.inner_dtype = inner_dtype;
  a.tol = tol;
  a.inner_tol = inner_tol;
  a.max_outer = max_outer;
  a.max_inner = max_inner;
  a.final_relres = final_relres;
  a.iters = iters;
  a.stream = (hipStream_t)stream;
  return DSLASH_OK;
}

// The workspace must be large enough and overlap none of the caller's arrays.
static int check_workspace(const dsl::SolveArgs& a, void* workspace, size_t ws_bytes, size_t need,
                           const void* U_lo) {
  if (!workspace || ws_bytes < need)
    return fail(DSLASH_E_WORKSPACE, "workspace needs %zu bytes, got %zu", need, workspace ? ws_bytes : size_t(0));
  const uint64_t vol = volume(a.dims);
  const size_t nspin = size_t(vol) * dsl::spinor_comps(a.op) * a.nv * 16;
  const size_t nlink = size_t(vol) * dsl::links_per_site(a.op) * 9 * 16;
  const size_t nlo = size_t(vol) * dsl::links_per_site(a.op) * 9 * dsl::dtype_bytes(a.inner_dtype);
  if (overlap(a.x64, nspin, workspace, need) || overlap(workspace, need, a.U64, nlink) ||
      overlap(workspace, need, a.b64, nspin))
    return fail(DSLASH_E_ALIAS, "x, b, U and workspace must not overlap");
  if (U_lo && (overlap(U_lo, nlo, workspace, need) || overlap(U_lo, nlo, a.x64, nspin)))
    return fail(DSLASH_E_ALIAS, "U_lo must not overlap x or the workspace");
  return DSLASH_OK;
}

size_t dslash_solve_workspace_bytes(const int dims[4], int Nc, int Nv, int inner_dtype) {
  if (check_geom(DSLASH_WILSON, dims, Nc, Nv) || !valid_inner(inner_dtype)) return 0;
  return dsl::solve_workspace_bytes(DSLASH_WILSON, dims, Nv, inner_dtype, false, false);
}

int dslash_solve(const void* U64, const void* U_lo, const void* b64, void* x64, const int dims[4], int Nc, int Nv,
                 double mass, int inner_dtype, double tol, double inner_tol, int max_outer, int max_inner,
                 void* workspace, size_t ws_bytes, double* final_relres, int* iters, void* stream) {
  g_err[0] = 0;
  dsl::SolveArgs a;
  if (int rc = solve_args(DSLASH_WILSON, U64, b64, x64, dims, Nc, Nv, mass, inner_dtype, tol, inner_tol, max_outer,
                          max_inner, final_relres, iters, stream, a))
    return rc;
  if (!U_lo) return fail(DSLASH_E_ARG, "U_lo is NULL");
  const size_t need = dsl::solve_workspace_bytes(DSLASH_WILSON, dims, Nv, inner_dtype, false, false);
  if (int rc = check_workspace(a, workspace, ws_bytes, need, U_lo)) return rc;
  a.U_lo = U_lo;
  a.workspace = workspace;
  return dsl::solve(a);
}

size_t dslash_solve_op_workspace_bytes(int op, const int dims[4], int Nc, int Nv, int inner_dtype) {
  if (check_geom(op, dims, Nc, Nv) || op == DSLASH_BRILLOUIN || !valid_inner(inner_dtype)) return 0;
  return dsl::solve_workspace_bytes(op, dims, Nv, inner_dtype);
}

int dslash_solve_op(int op, const void* U64, const void* b64, void* x64, const int dims[4], int Nc, int Nv,
                    double mass, int inner_dtype, double tol, double inner_tol, int max_outer, int max_inner,
                    void* workspace, size_t ws_bytes, double* final_relres, int* iters, void* stream) {
  g_err[0] = 0;
  dsl::SolveArgs a;
  if (int rc = solve_args(op, U64, b64, x64, dims, Nc, Nv, mass, inner_dtype, tol, inner_tol, max_outer, max_inner,
                          final_relres, iters, stream, a))
    return rc;
  const size_t need = dsl::solve_workspace_bytes(op, dims, Nv, inner_dtype);
  if (int rc = check_workspace(a, workspace, ws_bytes, need, nullptr)) return rc;
  a.workspace = workspace;
  return dsl::solve(a);
}

// ------------------------------------------------ solve without allocation
// dslash_solve_noalloc keeps its workspace in `scratch`, one static array per
// GPU that the library has run on, held until the process ends.  In host code
// the array's name is only a host-side stand-in: its device address is taken
// once per device with hipGetSymbolAddress (with that device current) and only
// that address reaches kernels and copies.
constexpr size_t kScratchBytes = DSLASH_SOLVE_NOALLOC_MAX_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
constexpr int kNoallocMaxNv = 256;

static int scratch_address(hipStream_t st, void** out) {
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  int dev = -1;
  hipError_t e = st ? hipStreamGetDevice(st, &dev) : hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "device of the stream");
  if (dev < 0 || dev >= kMaxDevices) return fail(DSLASH_E_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    int cur = -1;
    if ((e = hipGetDevice(&cur)) != hipSuccess) return hip_fail(e, "current device");
    if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return hip_fail(e, "select the stream's device");
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) {
      hipError_t e2 = hipSetDevice(cur);
      if (e == hipSuccess && e2 != hipSuccess) e = e2;
    }
    if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "scratch address");
    addr[dev] = p;
  }
  *out = addr[dev];
  return DSLASH_OK;
}

int dslash_solve_noalloc(const void* U64, const void* U_lo, const void* b64, void* x64, const int dims[4], int Nc,
                         int Nv, double mass, int inner_dtype, double tol, double inner_tol, int max_outer,
                         int max_inner, double* final_relres, int* iters, void* stream) {
  g_err[0] = 0;
  dsl::SolveArgs a;
  if (int rc = solve_args(DSLASH_WILSON, U64, b64, x64, dims, Nc, Nv, mass, inner_dtype, tol, inner_tol, max_outer,
                          max_inner, final_relres, iters, stream, a))
    return rc;
  if (!U_lo) return fail(DSLASH_E_ARG, "U_lo is NULL");
  if (Nv > kNoallocMaxNv) return fail(DSLASH_E_UNSUPPORTED, "at most %d right-hand sides (got %d)", kNoallocMaxNv, Nv);
  const size_t need = dsl::solve_workspace_bytes(DSLASH_WILSON, dims, Nv, inner_dtype, false, false);
  if (need > kScratchBytes)
    return fail(DSLASH_E_WORKSPACE, "the problem needs %zu bytes of workspace, the static scratch holds %zu", need,
                kScratchBytes);
  void* ws = nullptr;
  if (int rc = scratch_address(a.stream, &ws)) return rc;
  const uint64_t vol = volume(dims);
  const size_t nlo = size_t(vol) * 36 * dsl::dtype_bytes(inner_dtype);
  const size_t nspin = size_t(vol) * 12 * Nv * 16;
  if (overlap(U_lo, nlo, a.x64, nspin)) return fail(DSLASH_E_ALIAS, "U_lo must not overlap x");
  double host_d[dsl::kHostDoubles * kNoallocMaxNv];
  int host_i[dsl::kHostInts * kNoallocMaxNv];
  a.U_lo = U_lo;
  a.workspace = ws;
  a.host_d = host_d;
  a.host_i = host_i;
  return dsl::solve(a);
}

// ---------------------------------------------------------------- even-odd
static int check_even(const int dims[4]) {
  for (int i = 0; i < 4; ++i)
    if (dims[i] & 1) return fail(DSLASH_E_ARG, "even-odd form needs even extents (dims[%d] = %d)", i, dims[i]);
  return DSLASH_OK;
}

static int eo_copy_common(bool to_packed, const void* full, const void* even, const void* odd, const int dims[4],
                          size_t site_bytes, void* stream) {
  g_err[0] = 0;
  if (int rc = check_geom(DSLASH_WILSON, dims, 3, 1)) return rc;
  if (int rc = check_even(dims)) return rc;
  if (!full || !even || !odd) return fail(DSLASH_E_ARG, "NULL field pointer");
  if (site_bytes == 0 || site_bytes % 4) return fail(DSLASH_E_ARG, "site_bytes must be a positive multiple of 4");
  const size_t half = size_t(volume(dims) / 2) * site_bytes;
  if (overlap(full, 2 * half, even, half) || overlap(full, 2 * half, odd, half) || overlap(even, half, odd, half))
    return fail(DSLASH_E_ALIAS, "full, even and odd arrays must not overlap");
  const dsl::EoGeom e = dsl::make_eo_geom(dims, 1);
  hipError_t err = dsl::launch_eo_copy(to_packed, e, 0, to_packed ? full : even, to_packed ? (void*)even : (void*)full,
                                       site_bytes, (hipStream_t)stream);
  if (err == hipSuccess)
    err = dsl::launch_eo_copy(to_packed, e, 1, to_packed ? full : odd, to_packed ? (void*)odd : (void*)full,
                              site_bytes, (hipStream_t)stream);
  if (err != hipSuccess) return hip_fail(err, "dslash_eo copy launch");
  return DSLASH_OK;
}

int dslash_eo_pack(const void* full, void* even, void* odd, const int dims[4], size_t site_bytes, void* stream) {
  return eo_copy_common(true, full, even, odd, dims, site_bytes, stream);
}

int dslash_eo_unpack(const void* even, const void* odd, void* full, const int dims[4], size_t site_bytes,
                     void* stream) {
  return eo_copy_common(false, full, even, odd, dims, site_bytes, stream);
}

int dslash_eo_hop(const void* U_even, const void* U_odd, const void* in, void* out, const int dims[4], int Nc,
                  int Nv, int parity_out, int adjoint, int dtype, void* stream) {
  g_err[0] = 0;
  if (int rc = check_geom(DSLASH_WILSON, dims, Nc, Nv)) return rc;
  if (int rc = check_even(dims)) return rc;
  if (!valid_dtype(dtype)) return fail(DSLASH_E_ARG, "unknown dtype %d", dtype);
  if (parity_out != 0 && parity_out != 1) return fail(DSLASH_E_ARG, "parity_out must be 0 or 1 (got %d)", parity_out);
  if (!U_even || !U_odd || !in || !out) return fail(DSLASH_E_ARG, "NULL field pointer");
  const size_t eb = dsl::dtype_bytes(dtype);
  const size_t hspin = size_t(volume(dims) / 2) * 12 * Nv * eb, hlink = size_t(volume(dims) / 2) * 36 * eb;
  if (overlap(in, hspin, out, hspin)) return fail(DSLASH_E_ALIAS, "in and out overlap");
  if (overlap(U_even, hlink, out, hspin) || overlap(U_odd, hlink, out, hspin))
    return fail(DSLASH_E_ALIAS, "links and out overlap");
  const dsl::EoGeom e = dsl::make_eo_geom(dims, Nv);
  const void* Uo = parity_out == 0 ? U_even : U_odd;
  const void* Ui = parity_out == 0 ? U_odd : U_even;
  hipError_t err = dsl::launch_wilson_eo_hop(adjoint != 0, dtype, e, parity_out, Uo, Ui, in, out, nullptr, 0.0, 1.0,
                                             (hipStream_t)stream);
  if (err != hipSuccess) return hip_fail(err, "dslash_eo_hop launch");
  return DSLASH_OK;
}

size_t dslash_solve_eo_workspace_bytes(const int dims[4], int Nc, int Nv, int inner_dtype) {
  if (check_geom(DSLASH_WILSON, dims, Nc, Nv) || check_even(dims)) return 0;
  if (!valid_inner(inner_dtype)) return 0;
  return dsl::solve_workspace_bytes(DSLASH_WILSON, dims, Nv, inner_dtype, true);
}

int dslash_solve_eo(const void* U64, const void* b64, void* x64, const int dims[4], int Nc, int Nv, double m0,
                    int inner_dtype, double tol, double inner_tol, int max_outer, int max_inner, void* workspace,
                    size_t ws_bytes, double* final_relres, int* iters, void* stream) {
  g_err[0] = 0;
  dsl::SolveArgs a;
  if (int rc = solve_args(DSLASH_WILSON, U64, b64, x64, dims, Nc, Nv, m0, inner_dtype, tol, inner_tol, max_outer,
                          max_inner, final_relres, iters, stream, a))
    return rc;
  if (int rc = check_even(dims)) return rc;
  if (!(4.0 + m0 != 0.0)) return fail(DSLASH_E_ARG, "4 + m0 must be non-zero");
  const size_t need = dsl::solve_workspace_bytes(DSLASH_WILSON, dims, Nv, inner_dtype, true);
  if (int rc = check_workspace(a, workspace, ws_bytes, need, nullptr)) return rc;
  a.workspace = workspace;
  a.eo = true;
  return dsl::solve(a);
}

}  // extern "C"
