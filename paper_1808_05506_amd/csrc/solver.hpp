// Mixed-precision solver: host-side sequencing of dslash_solve and dslash_solve_eo.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace dsl {

struct SolveArgs {
  int op;
  const void* U64;
  const void* U_lo = nullptr;  // links in inner_dtype storage from the caller; null: converted into the workspace
  const void* b64;
  void* x64;
  int dims[4];
  int nv;
  double mass;
  int inner_dtype;
  double tol, inner_tol;
  int max_outer, max_inner;
  void* workspace;
  double* final_relres;
  int* iters;  // host, 2 * nv: inner iterations per column, then outer corrections per column
  hipStream_t stream;
  bool eo = false;  // inner solve on the even-site Schur complement (WILSON only)
  // host memory for the per-column values (kHostDoubles * nv doubles,
  // kHostInts * nv ints); null: the solve allocates its own
  double* host_d = nullptr;
  int* host_i = nullptr;
};

constexpr int kHostDoubles = 6, kHostInts = 2;

size_t solve_workspace_bytes(int op, const int dims[4], int nv, int inner_dtype, bool eo = false,
                             bool own_links = true);
int solve(const SolveArgs& a);
int set_error(int code, const char* msg);

}  // namespace dsl
