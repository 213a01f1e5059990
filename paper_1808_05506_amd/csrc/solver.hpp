// Mixed-precision solver: host-side sequencing of dslash_solve and dslash_solve_eo.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace dsl {

struct SolveArgs {
  int op;
  const void* U64;
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
  int* iters;
  hipStream_t stream;
  bool eo = false;  // inner solve on the even-site Schur complement (WILSON only)
};

size_t solve_workspace_bytes(int op, const int dims[4], int nv, int inner_dtype, bool eo = false);
int solve(const SolveArgs& a);
int set_error(int code, const char* msg);

}  // namespace dsl
