"""Python binding of ``libdslash.so`` (ctypes).

Argument marshalling only: shape, dtype, device and contiguity checks, then
one call into the C ABI (``include/dslash.h``) on the caller's current HIP
stream.  Every arithmetic step runs in the library's HIP kernels; there is no
host fallback, and a missing library raises at import of this module.

Tensor conventions (lattice dims = (Nx, Ny, Nz, Nt), site index slowest):

* links ``U``:  ``[Nt, Nz, Ny, Nx, 4, 3, 3]`` (Brillouin: ``[..., 40, 3, 3]``)
* Wilson / Brillouin spinors: ``[Nt, Nz, Ny, Nx, 4, 3, Nv]``
* staggered spinors: ``[Nt, Nz, Ny, Nx, 3, Nv]``
* complex64 / complex128 tensors, or for 16-bit storage real ``bfloat16`` /
  ``float16`` tensors with a trailing dimension 2 holding (re, im).
"""
from __future__ import annotations

import ctypes
import os

import torch

__all__ = [
    "STAGGERED", "WILSON", "BRILLOUIN", "DslashError", "library_path", "apply", "apply_adjoint",
    "backward", "brillouin_links", "convert", "solve", "dslash", "op_code", "clover_field", "eo_pack", "eo_unpack",
    "eo_hop", "compress_links", "apply_compressed", "brillouin_links_backward", "brillouin_links_autograd",
    "apply_brillouin_fly", "reload_tuning",
]

STAGGERED, WILSON, BRILLOUIN = 0, 1, 2
C64, C128, BF16, F16 = 0, 1, 2, 3

_HERE = os.path.dirname(os.path.abspath(__file__))


def library_path() -> str:
    return os.path.join(_HERE, "libdslash.so")


def _load():
    path = library_path()
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1808_05506_amd.build`")
    lib = ctypes.CDLL(path)
    vp, ip, i, d, sz = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    lib.dslash_apply.argtypes = [i, vp, vp, vp, ip, i, i, d, i, vp]
    lib.dslash_apply_adjoint.argtypes = [i, vp, vp, vp, ip, i, i, d, i, vp]
    lib.dslash_backward.argtypes = [i, vp, vp, vp, vp, vp, ip, i, i, d, i, vp]
    lib.dslash_brillouin_links.argtypes = [vp, vp, ip, i, i, vp]
    lib.dslash_convert.argtypes = [vp, i, vp, i, sz, vp]
    lib.dslash_solve_workspace_bytes.argtypes = [ip, i, i, i]
    lib.dslash_solve_workspace_bytes.restype = sz
    lib.dslash_solve.argtypes = [vp, vp, vp, vp, ip, i, i, d, i, d, d, i, i, vp, sz,
                                 ctypes.POINTER(ctypes.c_double), ip, vp]
    lib.dslash_solve_op_workspace_bytes.argtypes = [i, ip, i, i, i]
    lib.dslash_solve_op_workspace_bytes.restype = sz
    lib.dslash_solve_op.argtypes = [i, vp, vp, vp, ip, i, i, d, i, d, d, i, i, vp, sz,
                                    ctypes.POINTER(ctypes.c_double), ip, vp]
    lib.dslash_eo_pack.argtypes = [vp, vp, vp, ip, sz, vp]
    lib.dslash_eo_unpack.argtypes = [vp, vp, vp, ip, sz, vp]
    lib.dslash_eo_hop.argtypes = [vp, vp, vp, vp, ip, i, i, i, i, i, vp]
    lib.dslash_solve_eo_workspace_bytes.argtypes = [ip, i, i, i]
    lib.dslash_solve_eo_workspace_bytes.restype = sz
    lib.dslash_solve_eo.argtypes = [vp, vp, vp, ip, i, i, d, i, d, d, i, i, vp, sz,
                                    ctypes.POINTER(ctypes.c_double), ip, vp]
    lib.dslash_clover_field.argtypes = [vp, vp, ip, i, d, i, vp]
    lib.dslash_apply_clover.argtypes = [i, vp, vp, vp, vp, ip, i, i, d, i, i, vp]
    lib.dslash_compress_links.argtypes = [vp, vp, ip, i, i, vp]
    lib.dslash_apply_compressed.argtypes = [i, vp, vp, vp, ip, i, i, d, i, i, vp]
    lib.dslash_brillouin_links_backward.argtypes = [vp, vp, vp, vp, ip, i, i, vp]
    lib.dslash_brillouin_links_backward_workspace_bytes.argtypes = [ip, i, i]
    lib.dslash_brillouin_links_backward_workspace_bytes.restype = sz
    lib.dslash_brillouin_links_backward_ws.argtypes = [vp, vp, vp, vp, vp, sz, ip, i, i, vp]
    lib.dslash_apply_brillouin_fly.argtypes = [vp, vp, vp, ip, i, i, d, i, i, vp]
    lib.dslash_status_string.restype = ctypes.c_char_p
    lib.dslash_last_error.restype = ctypes.c_char_p
    for name in ("dslash_apply", "dslash_apply_adjoint", "dslash_backward", "dslash_brillouin_links",
                 "dslash_convert", "dslash_solve", "dslash_solve_op", "dslash_version", "dslash_eo_pack",
                 "dslash_eo_unpack", "dslash_eo_hop", "dslash_solve_eo", "dslash_clover_field", "dslash_apply_clover",
                 "dslash_compress_links", "dslash_apply_compressed", "dslash_brillouin_links_backward", "dslash_apply_brillouin_fly",
                 "dslash_reload_tuning", "dslash_brillouin_links_backward_ws"):
        getattr(lib, name).restype = ctypes.c_int
    return lib


_lib = _load()


class DslashError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = _lib.dslash_status_string(code).decode()
        detail = _lib.dslash_last_error().decode()
        super().__init__(f"{where}: {msg} ({detail})")


def _check(rc: int, where: str):
    if rc != 0:
        raise DslashError(rc, where)


def reload_tuning() -> None:
    """Re-read the DSLASH_* tuning variables from the environment (the
    library reads them once per process, at its first launch)."""
    _check(_lib.dslash_reload_tuning(), "dslash_reload_tuning")


def op_code(op) -> int:
    names = {"staggered": STAGGERED, "wilson": WILSON, "brillouin": BRILLOUIN}
    if isinstance(op, str):
        if op not in names:
            raise ValueError(f"unknown operator {op!r}")
        return names[op]
    if op in (STAGGERED, WILSON, BRILLOUIN):
        return int(op)
    raise ValueError(f"unknown operator {op!r}")


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.complex64:
        return C64
    if t.dtype == torch.complex128:
        return C128
    if t.dtype == torch.bfloat16 and t.shape[-1] == 2:
        return BF16
    if t.dtype == torch.float16 and t.shape[-1] == 2:
        return F16
    raise ValueError(f"unsupported tensor dtype {t.dtype} (shape {tuple(t.shape)})")


def _core_shape(t: torch.Tensor) -> tuple:
    """Shape without the trailing (re, im) axis of 16-bit storage."""
    return tuple(t.shape[:-1]) if _dtype_code(t) in (BF16, F16) else tuple(t.shape)


def _dims_c(shape) -> ctypes.Array:
    nt, nz, ny, nx = shape[:4]
    return (ctypes.c_int * 4)(nx, ny, nz, nt)


def _ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


def _stream(t: torch.Tensor):
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _require(t: torch.Tensor, name: str, like: torch.Tensor | None = None):
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch.Tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if like is not None and t.device != like.device:
        raise ValueError(f"{name} must be on {like.device}, not {t.device}")


def _spinor_shape(op: int, lat, nv: int) -> tuple:
    return tuple(lat) + ((3, nv) if op == STAGGERED else (4, 3, nv))


def _validate(op: int, U: torch.Tensor, psi: torch.Tensor):
    _require(U, "U")
    _require(psi, "psi")
    if _dtype_code(U) != _dtype_code(psi):
        raise ValueError(f"U and psi must have the same storage dtype ({U.dtype} vs {psi.dtype})")
    if U.device != psi.device:
        raise ValueError("U and psi must be on the same device")
    us, ps = _core_shape(U), _core_shape(psi)
    nl = 40 if op == BRILLOUIN else 4
    if len(us) != 7 or us[4:] != (nl, 3, 3):
        raise ValueError(f"U must have shape [Nt,Nz,Ny,Nx,{nl},3,3], got {us}")
    nv = ps[-1]
    if ps != _spinor_shape(op, us[:4], nv):
        raise ValueError(f"psi shape {ps} does not match U {us} for this operator")
    return us[:4], nv


def apply(op, U: torch.Tensor, psi: torch.Tensor, mass: float = 0.0, adjoint: bool = False,
          out: torch.Tensor | None = None, clover: torch.Tensor | None = None) -> torch.Tensor:
    """out = D psi (or D^dag psi), plus C psi for a clover field C from
    ``clover_field`` (WILSON, BRILLOUIN).  With gradients enabled and U or psi
    requiring them (and no ``out`` or ``clover``), this is the autograd
    operation ``dslash``: its backward returns (grad_U, grad_psi)."""
    if (out is None and clover is None and torch.is_grad_enabled()
            and (getattr(U, "requires_grad", False) or getattr(psi, "requires_grad", False))):
        return _DslashFn.apply(op_code(op), U, psi, float(mass), bool(adjoint))
    return _apply(op, U, psi, mass, adjoint, out, clover)


def _apply(op, U: torch.Tensor, psi: torch.Tensor, mass: float = 0.0, adjoint: bool = False,
           out: torch.Tensor | None = None, clover: torch.Tensor | None = None) -> torch.Tensor:
    op = op_code(op)
    lat, nv = _validate(op, U, psi)
    if out is None:
        out = torch.empty_like(psi)
    else:
        _require(out, "out", psi)
        if out.shape != psi.shape or out.dtype != psi.dtype:
            raise ValueError("out must match psi in shape and dtype")
    if clover is not None:
        _require(clover, "clover", psi)
        if _core_shape(clover) != tuple(lat) + (2, 18) or _dtype_code(clover) != _dtype_code(psi):
            raise ValueError(f"clover must be [Nt,Nz,Ny,Nx,2,18] in the dtype of psi, got {tuple(clover.shape)}")
        _check(_lib.dslash_apply_clover(op, _ptr(U), _ptr(clover), _ptr(psi), _ptr(out), _dims_c(lat), 3, nv,
                                        float(mass), int(bool(adjoint)), _dtype_code(psi), _stream(psi)),
               "dslash_apply_clover")
        return out
    fn = _lib.dslash_apply_adjoint if adjoint else _lib.dslash_apply
    _check(fn(op, _ptr(U), _ptr(psi), _ptr(out), _dims_c(lat), 3, nv, float(mass), _dtype_code(psi),
              _stream(psi)), "dslash_apply")
    return out


def apply_brillouin_fly(V: torch.Tensor, psi: torch.Tensor, mass: float = 0.0, adjoint: bool = False,
                        out: torch.Tensor | None = None) -> torch.Tensor:
    """D_B psi (or D_B^dag psi) with the off-axis links built from V inside the kernel."""
    lat, nv = _validate(WILSON, V, psi)   # V and psi have the shapes of the Wilson operator
    if out is None:
        out = torch.empty_like(psi)
    else:
        _require(out, "out", psi)
        if out.shape != psi.shape or out.dtype != psi.dtype:
            raise ValueError("out must match psi in shape and dtype")
    _check(_lib.dslash_apply_brillouin_fly(_ptr(V), _ptr(psi), _ptr(out), _dims_c(lat), 3, nv, float(mass),
                                           int(bool(adjoint)), _dtype_code(psi), _stream(psi)),
           "dslash_apply_brillouin_fly")
    return out


def compress_links(V: torch.Tensor) -> torch.Tensor:
    """First two rows of every SU(3) link: [Nt,Nz,Ny,Nx,4,2,3] (gauge compression)."""
    _require(V, "V")
    vs = _core_shape(V)
    if len(vs) != 7 or vs[4:] != (4, 3, 3):
        raise ValueError(f"V must have shape [Nt,Nz,Ny,Nx,4,3,3], got {vs}")
    pair = _dtype_code(V) in (BF16, F16)
    Vc = torch.empty(vs[:4] + (4, 2, 3) + ((2,) if pair else ()), dtype=V.dtype, device=V.device)
    _check(_lib.dslash_compress_links(_ptr(V), _ptr(Vc), _dims_c(vs), 3, _dtype_code(V), _stream(V)),
           "dslash_compress_links")
    return Vc


def apply_compressed(op, Vc: torch.Tensor, psi: torch.Tensor, mass: float = 0.0, adjoint: bool = False,
                     out: torch.Tensor | None = None) -> torch.Tensor:
    """out = D psi (or D^dag psi) for D_S or D_W with compressed links from ``compress_links``."""
    op = op_code(op)
    _require(Vc, "Vc")
    _require(psi, "psi", Vc)
    if _dtype_code(Vc) != _dtype_code(psi):
        raise ValueError("Vc and psi must have the same storage dtype")
    vs, ps = _core_shape(Vc), _core_shape(psi)
    if len(vs) != 7 or vs[4:] != (4, 2, 3):
        raise ValueError(f"Vc must have shape [Nt,Nz,Ny,Nx,4,2,3], got {vs}")
    nv = ps[-1]
    if op == BRILLOUIN or ps != _spinor_shape(op, vs[:4], nv):
        raise ValueError(f"psi shape {ps} does not match Vc {vs} for this operator")
    if out is None:
        out = torch.empty_like(psi)
    else:
        _require(out, "out", psi)
        if out.shape != psi.shape or out.dtype != psi.dtype:
            raise ValueError("out must match psi in shape and dtype")
    _check(_lib.dslash_apply_compressed(op, _ptr(Vc), _ptr(psi), _ptr(out), _dims_c(vs), 3, nv, float(mass),
                                        int(bool(adjoint)), _dtype_code(psi), _stream(psi)), "dslash_apply_compressed")
    return out


def clover_field(V: torch.Tensor, c_sw: float) -> torch.Tensor:
    """Packed clover term -(c_SW/2) sum sigma F of the links V: [Nt,Nz,Ny,Nx,2,18]."""
    _require(V, "V")
    vs = _core_shape(V)
    if len(vs) != 7 or vs[4:] != (4, 3, 3):
        raise ValueError(f"V must have shape [Nt,Nz,Ny,Nx,4,3,3], got {vs}")
    pair = _dtype_code(V) in (BF16, F16)
    C = torch.empty(vs[:4] + (2, 18) + ((2,) if pair else ()), dtype=V.dtype, device=V.device)
    _check(_lib.dslash_clover_field(_ptr(V), _ptr(C), _dims_c(vs), 3, float(c_sw), _dtype_code(V), _stream(V)),
           "dslash_clover_field")
    return C


def apply_adjoint(op, U, psi, mass: float = 0.0, out=None):
    return apply(op, U, psi, mass, adjoint=True, out=out)


def backward(op, U: torch.Tensor, grad_out: torch.Tensor, psi: torch.Tensor, mass: float = 0.0,
             need_grad_U: bool = True, need_grad_in: bool = True):
    """(grad_U, grad_in) of out = D[U] psi for upstream gradient grad_out."""
    op = op_code(op)
    lat, nv = _validate(op, U, psi)
    _require(grad_out, "grad_out", psi)
    if grad_out.shape != psi.shape or grad_out.dtype != psi.dtype:
        raise ValueError("grad_out must match psi in shape and dtype")
    gU = torch.empty_like(U) if need_grad_U else None
    gi = torch.empty_like(psi) if need_grad_in else None
    _check(_lib.dslash_backward(op, _ptr(U), _ptr(grad_out), _ptr(psi),
                                _ptr(gU) if gU is not None else None, _ptr(gi) if gi is not None else None,
                                _dims_c(lat), 3, nv, float(mass), _dtype_code(psi), _stream(psi)), "dslash_backward")
    return gU, gi


def brillouin_links(V: torch.Tensor) -> torch.Tensor:
    """Stored off-axis links W [Nt,Nz,Ny,Nx,40,3,3] of V (Tab. 1)."""
    _require(V, "V")
    vs = _core_shape(V)
    if len(vs) != 7 or vs[4:] != (4, 3, 3):
        raise ValueError(f"V must have shape [Nt,Nz,Ny,Nx,4,3,3], got {vs}")
    W = torch.empty(vs[:4] + (40, 3, 3), dtype=V.dtype, device=V.device)
    _check(_lib.dslash_brillouin_links(_ptr(V), _ptr(W), _dims_c(vs), 3, _dtype_code(V), _stream(V)),
           "dslash_brillouin_links")
    return W


def brillouin_links_backward(V: torch.Tensor, grad_W: torch.Tensor, W: torch.Tensor | None = None,
                             method: str | None = None) -> torch.Tensor:
    """Gradient with respect to V of Re sum conj(grad_W) W[V] (adjoint of ``brillouin_links``).
    W: optional ``brillouin_links(V)``.  method: "walk" walks every hop
    ordering through V (the only one without W); "subsets" sums the orderings
    of each path through the path averages of W; "levels" (the default with W)
    runs the first-hop recursion of the path averages backwards through a
    workspace of 756 words a site (when that allocation fails and no method
    was named, the sums through W run instead; they need none)."""
    auto = method is None
    if method is None:
        method = "walk" if W is None else "levels"
    if method not in ("walk", "subsets", "levels"):
        raise ValueError(f"method must be 'walk', 'subsets' or 'levels', got {method!r}")
    if (W is None) != (method == "walk"):
        raise ValueError(f"method {method!r} {'takes no' if method == 'walk' else 'needs'} W")
    _require(V, "V")
    _require(grad_W, "grad_W", V)
    vs = _core_shape(V)
    if len(vs) != 7 or vs[4:] != (4, 3, 3):
        raise ValueError(f"V must have shape [Nt,Nz,Ny,Nx,4,3,3], got {vs}")
    if tuple(grad_W.shape) != vs[:4] + (40, 3, 3) or grad_W.dtype != V.dtype or grad_W.device != V.device:
        raise ValueError("grad_W must be [Nt,Nz,Ny,Nx,40,3,3] in the dtype of V, on its device")
    if W is not None:
        _require(W, "W", V)
        if W.shape != grad_W.shape or W.dtype != V.dtype or W.device != V.device:
            raise ValueError("W must be brillouin_links(V): [Nt,Nz,Ny,Nx,40,3,3] in the dtype of V")
    gV = torch.empty_like(V)
    dims, code = _dims_c(vs), _dtype_code(V)
    if method == "levels":
        nbytes = _lib.dslash_brillouin_links_backward_workspace_bytes(dims, 3, code)
        if nbytes == 0:
            raise DslashError(f"dslash_brillouin_links_backward_workspace_bytes rejected dims {vs[:4]}")
        try:
            ws = torch.empty(nbytes, dtype=torch.uint8, device=V.device)
        except torch.cuda.OutOfMemoryError:
            if not auto:
                raise
            ws = None
    if method == "levels" and ws is not None:
        _check(_lib.dslash_brillouin_links_backward_ws(_ptr(V), _ptr(W), _ptr(grad_W), _ptr(gV), _ptr(ws), nbytes,
                                                       dims, 3, code, _stream(V)),
               "dslash_brillouin_links_backward_ws")
        return gV
    _check(_lib.dslash_brillouin_links_backward(_ptr(V), _ptr(W) if W is not None else None, _ptr(grad_W), _ptr(gV),
                                                dims, 3, code, _stream(V)),
           "dslash_brillouin_links_backward")
    return gV


class _BrillouinLinksFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, V):
        W = brillouin_links(V)
        ctx.save_for_backward(V, W)
        return W

    @staticmethod
    def backward(ctx, g):
        V, W = ctx.saved_tensors
        return brillouin_links_backward(V, g.contiguous(), W)


def brillouin_links_autograd(V: torch.Tensor) -> torch.Tensor:
    """Autograd-aware ``brillouin_links`` (complex64 / complex128)."""
    return _BrillouinLinksFn.apply(V)


_TORCH_OF = {C64: (torch.complex64, False), C128: (torch.complex128, False),
             BF16: (torch.bfloat16, True), F16: (torch.float16, True)}
_NAMES = {"c64": C64, "c128": C128, "bf16": BF16, "f16": F16}


def convert(x: torch.Tensor, dtype: str) -> torch.Tensor:
    """Copy x into storage ``dtype`` ('c64', 'c128', 'bf16', 'f16'), rounding to nearest even."""
    _require(x, "x")
    dst_code = _NAMES[dtype]
    src_code = _dtype_code(x)
    core = _core_shape(x)
    tdt, pair = _TORCH_OF[dst_code]
    out = torch.empty(core + ((2,) if pair else ()), dtype=tdt, device=x.device)
    n = 1
    for s in core:
        n *= s
    _check(_lib.dslash_convert(_ptr(x), src_code, _ptr(out), dst_code, n, _stream(x)), "dslash_convert")
    return out


def solve(op, U: torch.Tensor, b: torch.Tensor, mass: float, inner: str = "bf16", tol: float = 1e-10,
          inner_tol: float = 0.05, max_outer: int = 100, max_inner: int = 20000, x0: torch.Tensor | None = None,
          eo: bool = False, U_lo: torch.Tensor | None = None):
    """Solve D x = b by FP64 defect correction around a low-precision CG on D^dag D.

    U, b: complex128.  WILSON runs ``dslash_solve`` with the links in the inner
    storage ``U_lo`` (converted from U here when not given, so a caller solving
    repeatedly on one gauge field can convert once with ``convert``);
    STAGGERED runs ``dslash_solve_op``.  eo=True (WILSON only): the inner solve
    runs on the even-site Schur complement (``dslash_solve_eo``).  x0: initial
    guess, complex128 of b's shape on b's device (not modified).  Returns
    (x, info) with info = {relres: per-column FP64 ||b - D x||/||b||,
    inner_iters_per_column, outer_iters_per_column, inner_iters and
    outer_iters (their maxima over the columns), status}.  Raises ValueError
    on bad arguments before any library call; non-convergence is reported in
    info['status'] (5).
    """
    op = op_code(op)
    lat, nv = _validate(op, U, b)
    if U.dtype != torch.complex128:
        raise ValueError("solve takes complex128 links and right-hand sides")
    if op == BRILLOUIN:
        raise ValueError("the solver is built for STAGGERED and WILSON")
    if eo and op != WILSON:
        raise ValueError("the even-odd solve is built for WILSON only")
    if inner not in ("c64", "bf16", "f16"):
        raise ValueError(f"inner storage must be 'c64', 'bf16' or 'f16' (got {inner!r})")
    if x0 is not None:
        _require(x0, "x0")
        if x0.device != b.device or x0.dtype != torch.complex128 or x0.shape != b.shape:
            raise ValueError("x0 must be a complex128 tensor of b's shape on b's device")
    code = _NAMES[inner]
    use_lo = op == WILSON and not eo
    if U_lo is not None:
        if not use_lo:
            raise ValueError("U_lo is taken by the full-lattice Wilson solve only")
        _require(U_lo, "U_lo")
        if U_lo.device != U.device or _dtype_code(U_lo) != code or _core_shape(U_lo) != tuple(U.shape):
            raise ValueError(f"U_lo must be the links of U stored as {inner} on U's device")
    x = torch.zeros_like(b) if x0 is None else x0.clone()
    dims = _dims_c(lat)
    if eo:
        nbytes = _lib.dslash_solve_eo_workspace_bytes(dims, 3, nv, code)
    elif use_lo:
        nbytes = _lib.dslash_solve_workspace_bytes(dims, 3, nv, code)
    else:
        nbytes = _lib.dslash_solve_op_workspace_bytes(op, dims, 3, nv, code)
    if nbytes == 0:
        raise ValueError(f"unsupported solver configuration (inner={inner}, eo={eo})")
    if use_lo and U_lo is None:
        U_lo = convert(U, inner)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=b.device)
    relres = (ctypes.c_double * nv)()
    iters = (ctypes.c_int * (2 * nv))()
    rest = (dims, 3, nv, float(mass), code, float(tol), float(inner_tol), int(max_outer), int(max_inner), _ptr(ws),
            nbytes, relres, iters, _stream(b))
    if eo:
        name, rc = "dslash_solve_eo", _lib.dslash_solve_eo(_ptr(U), _ptr(b), _ptr(x), *rest)
    elif use_lo:
        name, rc = "dslash_solve", _lib.dslash_solve(_ptr(U), _ptr(U_lo), _ptr(b), _ptr(x), *rest)
    else:
        name, rc = "dslash_solve_op", _lib.dslash_solve_op(op, _ptr(U), _ptr(b), _ptr(x), *rest)
    if rc not in (0, 5):
        raise DslashError(rc, name)
    inner_cols, outer_cols = list(iters[:nv]), list(iters[nv:])
    return x, {"relres": list(relres), "inner_iters_per_column": inner_cols, "outer_iters_per_column": outer_cols,
               "inner_iters": max(inner_cols), "outer_iters": max(outer_cols), "status": rc}


def _site_bytes(t: torch.Tensor) -> int:
    per = 1
    for n in t.shape[4:]:
        per *= n
    return per * t.element_size()


def eo_pack(field: torch.Tensor):
    """(even, odd) packed halves [Nt][Nz][Ny][Nx/2][...] of a full-lattice field."""
    _require(field, "field")
    nt, nz, ny, nx = field.shape[:4]
    shape = (nt, nz, ny, nx // 2) + tuple(field.shape[4:])
    even = torch.empty(shape, dtype=field.dtype, device=field.device)
    odd = torch.empty_like(even)
    _check(_lib.dslash_eo_pack(_ptr(field), _ptr(even), _ptr(odd), _dims_c(field.shape), _site_bytes(field),
                               _stream(field)), "dslash_eo_pack")
    return even, odd


def eo_unpack(even: torch.Tensor, odd: torch.Tensor) -> torch.Tensor:
    """Full-lattice field from its packed even and odd halves."""
    _require(even, "even")
    _require(odd, "odd", even)
    if even.shape != odd.shape or even.dtype != odd.dtype:
        raise ValueError("even and odd halves must match in shape and dtype")
    nt, nz, ny, nh = even.shape[:4]
    full = torch.empty((nt, nz, ny, 2 * nh) + tuple(even.shape[4:]), dtype=even.dtype, device=even.device)
    _check(_lib.dslash_eo_unpack(_ptr(even), _ptr(odd), _ptr(full), _dims_c(full.shape), _site_bytes(even),
                                 _stream(even)), "dslash_eo_unpack")
    return full


def eo_hop(U_even: torch.Tensor, U_odd: torch.Tensor, psi: torch.Tensor, parity_out: int,
           adjoint: bool = False) -> torch.Tensor:
    """H psi on the packed sites of parity parity_out; psi packed on the other parity."""
    for t, n in ((U_even, "U_even"), (U_odd, "U_odd"), (psi, "psi")):
        _require(t, n, U_even)
    cs = _core_shape(psi)
    if len(cs) != 7 or cs[4:6] != (4, 3):
        raise ValueError(f"psi must be packed [Nt,Nz,Ny,Nx/2,4,3,Nv], got {cs}")
    if _core_shape(U_even) != cs[:4] + (4, 3, 3) or U_odd.shape != U_even.shape:
        raise ValueError("U_even/U_odd must be packed [Nt,Nz,Ny,Nx/2,4,3,3] matching psi")
    if _dtype_code(U_even) != _dtype_code(psi) or _dtype_code(U_odd) != _dtype_code(psi):
        raise ValueError("links and psi must share the storage dtype")
    nt, nz, ny, nh = cs[:4]
    out = torch.empty_like(psi)
    dims = (ctypes.c_int * 4)(2 * nh, ny, nz, nt)
    _check(_lib.dslash_eo_hop(_ptr(U_even), _ptr(U_odd), _ptr(psi), _ptr(out), dims, 3, cs[6], int(parity_out),
                              int(bool(adjoint)), _dtype_code(psi), _stream(psi)), "dslash_eo_hop")
    return out


class _DslashFn(torch.autograd.Function):
    """out = D[U] psi (or D^dag psi) with the hand-written backward of the library.

    Forward op:  grad_psi = D^dag g,  grad_U = link gradient of Re<g, D psi>.
    Adjoint op:  Re<g, D^dag psi> = Re<psi, D g>, so grad_psi = D g and
                 grad_U = link gradient with the roles of g and psi swapped.
    """

    @staticmethod
    def forward(ctx, op, U, psi, mass, adjoint):
        ctx.op, ctx.mass, ctx.adjoint = op, mass, adjoint
        ctx.save_for_backward(U, psi)
        return _apply(op, U, psi, mass, adjoint)

    @staticmethod
    def backward(ctx, g):
        U, psi = ctx.saved_tensors
        g = g.contiguous()
        need_u, need_psi = ctx.needs_input_grad[1], ctx.needs_input_grad[2]
        gU = gpsi = None
        if not ctx.adjoint:
            gU, gpsi = backward(ctx.op, U, g, psi, ctx.mass, need_u, need_psi)
        else:
            if need_u:
                gU, _ = backward(ctx.op, U, psi, g, ctx.mass, True, False)
            if need_psi:
                gpsi = _apply(ctx.op, U, g, ctx.mass, adjoint=False)
        return None, gU, gpsi, None, None


def dslash(op, U: torch.Tensor, psi: torch.Tensor, mass: float = 0.0, adjoint: bool = False) -> torch.Tensor:
    """Autograd-aware D psi (complex64 / complex128).  BRILLOUIN: U is the stored W;
    combine with ``brillouin_links_autograd`` for the gradient with respect to V."""
    return _DslashFn.apply(op_code(op), U, psi, float(mass), bool(adjoint))
