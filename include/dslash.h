/*
 * dslash.h -- C ABI of the MI355X (gfx950) Dirac-operator library.
 *
 * The library applies three lattice Dirac operators to a block of N_v
 * right-hand-side vectors, following S. Duerr, "Three Dirac operators on two
 * architectures with one piece of code and no hassle" (LATTICE 2018):
 *
 *   STAGGERED  D_S  (Sec. 3, the D_S equation; eta phases, precomputed links V)
 *   WILSON     D_W  (Sec. 4, eq. def_wils at c_SW = 0)
 *   BRILLOUIN  D_B  (Sec. 5, eqs. def_bril, def_der, def_lap at c_SW = 0, with
 *                    the precomputed off-axis links W of Tab. 1)
 *
 * plus the adjoint operators, the link gradient (backward pass) of
 * L = Re sum chi^dag D psi, the construction of W from V, and a
 * mixed-precision solver for D x = b.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * dims      {Nx, Ny, Nz, Nt}, the paper's index order (Sec. 2).  Periodic
 *           boundaries in all four directions.  Site index
 *           s = x + Nx*(y + Ny*(z + Nz*t)), 0-based coordinates.
 * Nc        number of colours; only 3 is built.
 * Nv        number of right-hand sides, >= 1.
 * dtype     storage of every field argument of the call:
 *             DSLASH_C64  complex float  (re, im) interleaved, FP32 arithmetic
 *             DSLASH_C128 complex double (re, im) interleaved, FP64 arithmetic
 *             DSLASH_BF16 bfloat16 pairs (re, im), FP32 arithmetic
 *             DSLASH_F16  IEEE half pairs (re, im), FP32 arithmetic
 *           Low-precision stores round to nearest even.
 * Layouts   (C order, site index slowest, as the paper's Fortran arrays with
 *           the space-time index right-most, Sec. 2):
 *             links V     [Nt][Nz][Ny][Nx][4][Nc][Nc], element [..][mu][a][b]
 *                         = (V_mu(x))_{ab}, mu = 0..3 for x, y, z, t
 *             off-axis W  [Nt][Nz][Ny][Nx][40][Nc][Nc] (Tab. 1 caption); the
 *                         direction d in {-1,0,1}^4 with highest-index non-zero
 *                         component +1 sits in slot n(d) - 41,
 *                         n(d) = sum_mu (d_mu + 1) 3^mu; the other 40 follow
 *                         from W_{-d}(x) = W_d(x-d)^dag
 *             Wilson and Brillouin spinor block  [Nt][Nz][Ny][Nx][4][Nc][Nv]
 *             staggered spinor block             [Nt][Nz][Ny][Nx][Nc][Nv]
 *           (the paper's vec(Nv,Nc,4,...) and suv(Nv,Nc,...) options).
 * gamma     Euclidean chiral basis: gamma_k = [[0, -i sigma_k], [i sigma_k, 0]]
 *           (k = 1,2,3), gamma_4 = [[0, 1], [1, 0]], gamma_5 = diag(1,1,-1,-1).
 * Pointers  all field pointers are DEVICE pointers owned by the caller; the
 *           library allocates nothing in apply / adjoint / backward / links.
 *           Outputs are overwritten, never accumulated into.
 * stream    a hipStream_t passed as void* (NULL = the default stream).  Every
 *           call except dslash_solve is asynchronous on it.
 * Errors    return codes, never exceptions or aborts.  Arguments are checked
 *           synchronously before any launch; a failed call launches nothing.
 *           dslash_last_error() gives a thread-local detail string.
 */
#ifndef DSLASH_H
#define DSLASH_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DSLASH_OK = 0,
  DSLASH_E_ARG = 1,          /* null pointer, bad dims / Nv / op / dtype        */
  DSLASH_E_UNSUPPORTED = 2,  /* Nc != 3, or an op/dtype pair that is not built  */
  DSLASH_E_ALIAS = 3,        /* an output aliases an input                      */
  DSLASH_E_HIP = 4,          /* a HIP runtime call or launch failed             */
  DSLASH_E_NOCONV = 5,       /* solver hit its iteration limit                  */
  DSLASH_E_WORKSPACE = 6     /* solver workspace null or too small              */
} dslash_status;

typedef enum { DSLASH_STAGGERED = 0, DSLASH_WILSON = 1, DSLASH_BRILLOUIN = 2 } dslash_op;

typedef enum { DSLASH_C64 = 0, DSLASH_C128 = 1, DSLASH_BF16 = 2, DSLASH_F16 = 3 } dslash_dtype;

/*
 * out = D in.
 *   STAGGERED (Sec. 3):  out(x) = m in(x) + sum_mu eta_mu(x)/2 [V_mu(x) in(x+mu)
 *                                  - V_mu(x-mu)^dag in(x-mu)],
 *                        eta_1 = 1, eta_2 = (-1)^x, eta_3 = (-1)^(x+y),
 *                        eta_4 = (-1)^(x+y+z); mass = m (0 is the paper's
 *                        operator).  Every extent must be even.
 *   WILSON (eq. def_wils, c_SW = 0):  D_W = sum gamma_mu nabla^std_mu
 *                        - Laplace^std / 2 + m0, V_{-mu}(x) = V_mu(x-mu)^dag;
 *                        mass = m0.  U = V.
 *   BRILLOUIN (eq. def_bril, c_SW = 0):  D_B = sum gamma_mu nabla^iso_mu
 *                        - Laplace^bri / 2 + m0 with the 54-point derivative
 *                        (eq. def_der) and 81-point Laplacian (eq. def_lap);
 *                        mass = m0.  U = the stored W.
 * U, in: read only.  out: written once per element.  in == out -> E_ALIAS.
 * Every extent >= 2 (>= 3 is needed for the Brillouin stencil to be distinct
 * sites, but 2 is accepted and sums coinciding terms).
 */
int dslash_apply(int op, const void* U, const void* in, void* out, const int dims[4], int Nc, int Nv,
                 double mass, int dtype, void* stream);

/*
 * out = D^dag in.  STAGGERED: the hop term changes sign (it is
 * anti-Hermitian; the mass is real).  WILSON, BRILLOUIN: gamma_5 D gamma_5,
 * i.e. every gamma_mu in the hop terms changes sign.  Same arguments and
 * errors as dslash_apply.
 */
int dslash_apply_adjoint(int op, const void* U, const void* in, void* out, const int dims[4], int Nc,
                         int Nv, double mass, int dtype, void* stream);

/*
 * Clover term (eqs. def_wils and def_bril, the term -(c_SW/2) sum_{mu<nu}
 * sigma_{mu nu} F_{mu nu}(x) delta_{x,y}; the paper benchmarks c_SW = 0 and
 * defines neither sigma nor F).  Built as
 *   sigma_{mu nu} = (i/2) [gamma_mu, gamma_nu]   (chiral basis, as for D_W),
 *   F_{mu nu}(x)  = (Q_{mu nu}(x) - Q_{mu nu}(x)^dag) / (8 i),
 * Q_{mu nu}(x) = the four plaquettes of the (mu, nu) plane starting and
 * ending at x, each run x -> x+a -> x+a+b -> x+b -> x for (a, b) = (mu, nu),
 * (nu, -mu), (-mu, -nu), (-nu, mu); no trace subtraction.  The term is
 * Hermitian and block diagonal: block b acts on spins 2b, 2b+1 with row index
 * 3 s' + c.
 *
 * C (output): [Nt][Nz][Ny][Nx][2][18] storage words; per block the real
 * diagonal pairwise as (H_00, H_11), (H_22, H_33), (H_44, H_55) in (re, im),
 * then the upper triangle H_ij, i < j, row by row.  Same storage dtype as V
 * (36 words per site, the size of the links).  V: [..][4][3][3], read only.
 * V and C must not overlap (E_ALIAS).  Asynchronous on `stream`.
 */
int dslash_clover_field(const void* V, void* C, const int dims[4], int Nc, double c_sw, int dtype,
                        void* stream);

/*
 * out = (D + C) in, or (D^dag + C) in if adjoint != 0 (C is Hermitian), for
 * op = WILSON (U = V) or BRILLOUIN (U = the stored W), with C from
 * dslash_clover_field (same dtype).  Other ops -> E_ARG; C == NULL -> E_ARG;
 * otherwise the arguments and errors of dslash_apply, and out must not
 * overlap C (E_ALIAS).  N_v = 12 with FP32 arithmetic runs the row-staged
 * kernels with the term fused into their last step.
 */
int dslash_apply_clover(int op, const void* U, const void* C, const void* in, void* out, const int dims[4],
                        int Nc, int Nv, double mass, int adjoint, int dtype, void* stream);

/*
 * Adjoint of dslash_brillouin_links (Tab. 1): grad_V = dR/dV for
 * R = Re sum conj(grad_W) W[V], i.e. the chain rule through every path
 * product of every stored W_d.  For a path product M = A_1 ... A_k in the
 * mean over the k! hop orderings, hop i receives P^dag grad_W Q^dag / k!
 * (P, Q the products before and after it), or the adjoint of that for a hop
 * against the link (A_i = V_mu(y - mu)^dag).  Together with the BRILLOUIN
 * branch of dslash_backward this is the link gradient of D_B with respect to
 * V.  V: [..][4][3][3]; W (nullable): dslash_brillouin_links(V), the stored
 * off-axis links of the same V -- with it the orderings that share the hops
 * before and after hop i are summed at once as |S|! |R|! W_S^dag grad_W W_R^dag
 * (W_S, W_R the path averages of the sub-displacements), without it every
 * ordering is walked through V; grad_W: [..][40][3][3]; grad_V: [..][4][3][3]
 * (written, deterministic: no atomics).  C64 and C128 only.  grad_V must not
 * overlap V, W or grad_W (E_ALIAS).  Asynchronous on `stream`.
 */
int dslash_brillouin_links_backward(const void* V, const void* W, const void* grad_W, void* grad_V, const int dims[4],
                                    int Nc, int dtype, void* stream);

/*
 * Workspace bytes dslash_brillouin_links_backward_ws needs: vol * 756
 * complex words of dtype (grad_W and W, 360 words a site each, and V, 36, as
 * structures of arrays); 0 on bad arguments.
 */
size_t dslash_brillouin_links_backward_workspace_bytes(const int dims[4], int Nc, int dtype);

/*
 * The gradient of dslash_brillouin_links_backward, computed through the
 * recursion of the path averages by their first hop (Tab. 1):
 *   W_d(x) = (1/k) sum_{mu: d_mu != 0} A(x) W_{d - d_mu mu}(x + d_mu mu),
 * A = V_mu(x) for d_mu = +1, V_mu(x - mu)^dag for d_mu = -1, W_0 = 1.
 * Reverse mode runs from the four-hop directions down: the total gradient of
 * each stored direction with one to three hops (its grad_W entry plus what the
 * directions with one more hop pass to it) goes to `workspace`, then every
 * link gathers its share from the totals and the path averages in W.  The
 * workspace holds these arrays with word e of slot j at [(j * 9 + e) * vol +
 * site], so consecutive sites read consecutive words.  Same
 * result as dslash_brillouin_links_backward up to rounding order, with about a
 * fifth of the matrix products; deterministic (gathers in a fixed order, no
 * atomics).  V, grad_W, grad_V as there; W: dslash_brillouin_links(V),
 * required; workspace: 16-byte aligned device memory of ws_bytes >=
 * dslash_brillouin_links_backward_workspace_bytes (else E_ARG), overwritten,
 * owned by the caller, must not overlap any other argument (E_ALIAS).  C64
 * and C128 only.  Asynchronous on `stream`.
 */
int dslash_brillouin_links_backward_ws(const void* V, const void* W, const void* grad_W, void* grad_V, void* workspace,
                                       size_t ws_bytes, const int dims[4], int Nc, int dtype, void* stream);

/*
 * out = D_B in (adjoint == 0) or D_B^dag in, with the off-axis links W_d(x)
 * built from the one-hop links V inside the kernel for every hop (Tab. 1; the
 * paper's variant without a precomputed W, Sec. 5): no W array is read or
 * stored.  V: [..][4][3][3].  Built for N_v = 4, 8, 12, 16 and 24, C64
 * storage and the x-extents the row-staged FP32 kernel covers (rows of at
 * least 12 sites at N_v = 12); E_UNSUPPORTED otherwise.  Other arguments and
 * errors as dslash_apply.
 */
int dslash_apply_brillouin_fly(const void* V, const void* in, void* out, const int dims[4], int Nc, int Nv,
                               double mass, int adjoint, int dtype, void* stream);

/*
 * Gauge compression (Sec. 4 names storing N_c - 1 colour rows of V as a next
 * step; Sec. 5 notes that 36 of the 40 W are not special unitary, so it is
 * offered for V only).  An SU(3) link is fixed by its first two rows: the
 * third is u_2j = conj(u_0k u_1l - u_0l u_1k), (j, k, l) cyclic.
 *
 * dslash_compress_links: Vc[..][mu][a][b] = V[..][mu][a][b] for a = 0, 1;
 * Vc is [Nt][Nz][Ny][Nx][4][2][3] (24 words per site instead of 36).  V must
 * be SU(3) for the compressed operator to equal the full one; nothing checks
 * this.  V and Vc must not overlap (E_ALIAS).  Asynchronous on `stream`.
 */
int dslash_compress_links(const void* V, void* Vc, const int dims[4], int Nc, int dtype, void* stream);

/*
 * out = D in (adjoint == 0) or D^dag in, for op = STAGGERED or WILSON, with
 * the links read from their compressed form Vc and completed in the kernel.
 * Other ops -> E_ARG; otherwise the arguments and errors of dslash_apply.
 * N_v = 12 runs the row-staged kernels (STAGGERED: C64, C128; WILSON: FP32
 * arithmetic on C64, BF16, F16 storage).
 */
int dslash_apply_compressed(int op, const void* Vc, const void* in, void* out, const int dims[4], int Nc,
                            int Nv, double mass, int adjoint, int dtype, void* stream);

/*
 * Backward pass of out = D[U] in for a real loss L with grad_out = dL/dout
 * (PyTorch convention for complex tensors: dL/dRe + i dL/dIm).
 *   grad_in = D^dag grad_out                                   (nullable)
 *   grad_U  = G,  G_mu(x) = sum_v sum_s [ g(x)_s (x) conj((P_+ in(x+mu))_s)
 *                                  + (P_- in(x))_s (x) conj(g(x+mu)_s) ]  (nullable)
 * with (x) the colour outer product, g = grad_out, and P_+, P_- the spin
 * factors of the forward and backward hop: eta_mu(x)/2 and -eta_mu(x)/2 for
 * STAGGERED, -(1 - gamma_mu)/2 and -(1 + gamma_mu)/2 for WILSON.  This is the
 * link gradient of L = Re sum conj(grad_out) * (D in) with the links treated
 * as free complex matrices.  grad_U has the layout of V.  BRILLOUIN (U = the
 * stored W, taken as free matrices): grad_U has the layout of W and
 *   G_{W_d}(x) = sum_v sum_s [ (S_d g(x))_s (x) conj(in(x+d)_s)
 *                            + in(x)_s (x) conj((S_{-d} g(x+d))_s) ]
 * for every stored d, S_d = -lambda_k/2 + rho_k d.gamma the spin factor of the
 * hop d (eqs. def_der, def_lap; W_d(x) also enters out(x+d) as W_{-d}(x+d)^dag).
 * The gradient with respect to V follows from dslash_brillouin_links_backward.
 * Outputs may not alias inputs (E_ALIAS).  Only C64 and C128 are accepted.
 */
int dslash_backward(int op, const void* U, const void* grad_out, const void* in, void* grad_U,
                    void* grad_in, const int dims[4], int Nc, int Nv, double mass, int dtype,
                    void* stream);

/*
 * W = off-axis links of V (Tab. 1): for each of the 40 stored directions d
 * with k non-zero components, W_d(x) = (1/k!) sum over the k! orderings of
 * the hops of the ordered product of V along the path from x, with
 * V_{-mu}(y) = V_mu(y - mu)^dag.  V [..][4][Nc][Nc] -> W [..][40][Nc][Nc].
 * Built level by level from the same mean grouped by the first hop,
 * W_d(x) = (1/k) sum_{mu: d_mu != 0} V_{d_mu mu}(x) W_{d - d_mu mu}(x + d_mu mu),
 * each level reading the one below from W (k products for a k-hop direction).
 * C64 or C128.  V and W must not overlap (E_ALIAS).
 */
int dslash_brillouin_links(const void* V, void* W, const int dims[4], int Nc, int dtype, void* stream);

/*
 * Copy n complex numbers from src (src_dtype) to dst (dst_dtype), rounding to
 * nearest even when narrowing.  Any pair of the four dtypes.  n == 0 is a
 * no-op.  src == dst -> E_ALIAS.
 */
int dslash_convert(const void* src, int src_dtype, void* dst, int dst_dtype, size_t n, void* stream);

/*
 * Workspace bytes dslash_solve needs for this problem (0 on bad arguments).
 */
size_t dslash_solve_workspace_bytes(const int dims[4], int Nc, int Nv, int inner_dtype);

/*
 * Solve D_W x = b for all Nv right-hand sides (the paper has no solver; this
 * is the mixed-precision scheme of FP64 defect correction around an inner CG
 * on the normal equations D_W^dag D_W e = D_W^dag r, for the Wilson operator
 * of eq. def_wils at c_SW = 0).
 *   Outer loop, FP64 on the GPU:  r = b - D_W x, relres_v = ||r_v|| / ||b_v||;
 *     stop when every relres_v <= tol.
 *   Inner loop: CG on D_W^dag D_W with links and vectors stored in inner_dtype
 *     (C64, BF16 or F16) and FP32 arithmetic, the right-hand side r scaled
 *     per column to unit RMS, run to inner_tol (relative, per column) or
 *     max_inner iterations; then x += scale * e in FP64.
 *   Inner products and norms are accumulated in FP64 in a fixed order.
 * U64, b64: C128 device arrays (links [..][4][3][3], spinors [..][4][3][Nv]);
 * U_lo: the same links stored in inner_dtype (e.g. from dslash_convert), read
 * only, so repeated solves on one gauge field convert the links once; x64:
 * C128 device array holding the initial guess on entry and the solution on
 * exit.  workspace: device memory of at least dslash_solve_workspace_bytes
 * bytes, owned by the caller.  x may not overlap b, U64, U_lo or the
 * workspace (E_ALIAS).
 * final_relres (host, Nv doubles, nullable): true FP64 relative residuals.
 * iters (host, 2 * Nv ints, nullable): iters[v] = inner iterations run on
 * column v, iters[Nv + v] = outer corrections applied to column v.
 * Synchronises the stream.  Returns E_NOCONV (x still updated) if max_outer
 * outer iterations did not reach tol.
 */
int dslash_solve(const void* U64, const void* U_lo, const void* b64, void* x64, const int dims[4], int Nc, int Nv,
                 double mass, int inner_dtype, double tol, double inner_tol, int max_outer, int max_inner,
                 void* workspace, size_t ws_bytes, double* final_relres, int* iters, void* stream);

/*
 * dslash_solve for op = STAGGERED (Sec. 3) or WILSON, taking only the FP64
 * links: the inner_dtype copy of the links is made in the workspace on every
 * call.  Arguments and results as dslash_solve; op = BRILLOUIN -> E_ARG.
 */
size_t dslash_solve_op_workspace_bytes(int op, const int dims[4], int Nc, int Nv, int inner_dtype);
int dslash_solve_op(int op, const void* U64, const void* b64, void* x64, const int dims[4], int Nc, int Nv,
                    double mass, int inner_dtype, double tol, double inner_tol, int max_outer, int max_inner,
                    void* workspace, size_t ws_bytes, double* final_relres, int* iters, void* stream);

/*
 * dslash_solve for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same solve, the same arguments and results, with no workspace argument.
 * Its workspace is a static device array of DSLASH_SOLVE_NOALLOC_MAX_BYTES
 * bytes inside the library, one per GPU the library runs on, held until the
 * process ends; the call allocates nothing (no hipMalloc, hipFree or
 * allocating library routine, no host heap memory).  Problems whose workspace
 * (dslash_solve_workspace_bytes) exceeds the array, or with Nv > 256, return
 * E_WORKSPACE / E_UNSUPPORTED before any launch.  Every call on one GPU shares
 * that GPU's array and leaves its contents behind (the solve initialises all
 * it reads): calls that overlap on one GPU -- on different streams or from
 * different host threads -- race and must be serialised by the caller.
 * Synchronises the stream, so it cannot itself be captured into a graph.
 */
#define DSLASH_SOLVE_NOALLOC_MAX_BYTES ((size_t)128 << 20)
int dslash_solve_noalloc(const void* U64, const void* U_lo, const void* b64, void* x64, const int dims[4], int Nc,
                         int Nv, double mass, int inner_dtype, double tol, double inner_tol, int max_outer,
                         int max_inner, double* final_relres, int* iters, void* stream);

/*
 * Even-odd (checkerboard) form of D_W, the eo-decomposition named as a next
 * tuning step at the end of Sec. 4.  All four extents must be even (E_ARG
 * otherwise).  parity(x) = (x + y + z + t) mod 2; every hop of D_W joins
 * opposite parities, so D_W = [[A, H_eo], [H_oe, A]] with A = 4 + m0 and
 *   H in(x) = -1/2 sum_mu [(1 - gamma_mu) V_mu(x) in(x+mu) + (1 + gamma_mu) V_mu(x-mu)^dag in(x-mu)].
 * Packed layout of one parity p: [Nt][Nz][Ny][Nx/2][...], the packed index
 * i of row (y, z, t) holding x = 2 i + ((p + y + z + t) mod 2).
 *
 * dslash_eo_pack: split a full-lattice array with site_bytes bytes per site
 * (e.g. 12 Nc Nv or 4 Nc Nc storage words) into its even and odd packed
 * halves; dslash_eo_unpack is the inverse.  No arithmetic; any dtype (the
 * caller states the bytes).  Outputs may not overlap inputs (E_ALIAS).
 */
int dslash_eo_pack(const void* full, void* even, void* odd, const int dims[4], size_t site_bytes, void* stream);
int dslash_eo_unpack(const void* even, const void* odd, void* full, const int dims[4], size_t site_bytes,
                     void* stream);

/*
 * out = H in restricted to output parity `parity_out` (0 or 1): in is a
 * packed field of parity 1 - parity_out, out a packed field of parity
 * parity_out, both [..][Nx/2][4][Nc][Nv].  U_even, U_odd: the links V packed
 * by parity ([..][Nx/2][4][Nc][Nc] each; V_mu(x) of the forward hops comes
 * from the output parity, V_mu(x - mu) of the backward hops from the other).
 * adjoint != 0: gamma_mu -> -gamma_mu (H^dag = gamma_5 H gamma_5).  Any dtype;
 * in == out -> E_ALIAS.
 */
int dslash_eo_hop(const void* U_even, const void* U_odd, const void* in, void* out, const int dims[4], int Nc,
                  int Nv, int parity_out, int adjoint, int dtype, void* stream);

/* Workspace bytes dslash_solve_eo needs (0 on bad arguments). */
size_t dslash_solve_eo_workspace_bytes(const int dims[4], int Nc, int Nv, int inner_dtype);

/*
 * Solve D_W x = b as dslash_solve(WILSON, ...) does -- the same FP64 outer
 * defect correction on the full lattice, the same arguments and results --
 * with the inner solve on the even-site Schur complement
 *   M = A - H_eo A^-1 H_oe:   M e_e = rhat_e - H_eo A^-1 rhat_o  (CG on M^dag M),
 *   e_o = A^-1 (rhat_o - H_oe e_e),
 * in inner_dtype storage (C64, BF16 or F16) with FP32 arithmetic; the links
 * are converted and packed in the workspace.  iters: 2 * Nv ints as for
 * dslash_solve.  All extents must be even.  Synchronises the stream.
 */
int dslash_solve_eo(const void* U64, const void* b64, void* x64, const int dims[4], int Nc, int Nv, double m0,
                    int inner_dtype, double tol, double inner_tol, int max_outer, int max_inner, void* workspace,
                    size_t ws_bytes, double* final_relres, int* iters, void* stream);

/* Human-readable name of a status code (static string). */
const char* dslash_status_string(int status);

/* Thread-local detail of the last failure in this thread ("" if none). */
const char* dslash_last_error(void);

/* ABI version (major*100 + minor). */
int dslash_version(void);

/*
 * Re-reads the tuning variables DSLASH_<NAME> (chunk length, prefetch depth,
 * t steps per workgroup, buffer scheme, kernel family, ...) from the
 * environment.  They are read once per process, at the first launch that
 * consults them; a caller that changes them later (a tuning sweep, a test of
 * each kernel form) calls this afterwards.  Not to be called while another
 * thread launches.  Returns DSLASH_OK.
 */
int dslash_reload_tuning(void);

#ifdef __cplusplus
}
#endif

#endif /* DSLASH_H */
