"""Python binding of the C ABI (argument marshalling only).

Every numerical step runs in libmpid's HIP kernels; PyTorch provides device
memory and the current stream.  Matrices cross the boundary column-major: a
column-major m x n tensor is the transpose of a contiguous (n, m) tensor.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib

C = _lib.C

PREC = {
    "f64": C["ID_PREC_F64"],
    "mixed_f16": C["ID_PREC_MIXED_F16"],
    "mixed_bf16": C["ID_PREC_MIXED_BF16"],
    "mixed_bf16x3": C["ID_PREC_MIXED_BF16X3"],
    "mixed_f32": C["ID_PREC_MIXED_F32"],
}
RULE = {"pivot_rel": C["ID_RANK_PIVOT_REL"], "frob_rel": C["ID_RANK_FROB_REL"]}
DTYPE = {torch.float32: C["ID_F32"], torch.float64: C["ID_F64"]}


def colmajor(A: torch.Tensor):
    """(A', lda): A' is A itself when already column-major, else a column-major copy."""
    if A.dim() != 2:
        raise ValueError("expected a matrix")
    if A.dtype not in DTYPE:
        raise TypeError("A must be float32 or float64")
    m, n = A.shape
    if A.stride(0) == 1 and (n <= 1 or A.stride(1) >= max(m, 1)):
        return A, max(A.stride(1) if n > 1 else m, m, 1)
    Ac = A.t().contiguous().t()
    return Ac, max(m, 1)


def empty_colmajor(rows: int, cols: int, dtype=torch.float64, device=None, zero=False):
    """A column-major rows x cols tensor (leading dimension max(rows, 1))."""
    f = torch.zeros if zero else torch.empty
    return f((cols, max(rows, 1)), dtype=dtype, device=device).t()[:rows]


def _stream(device=None):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


ROUND = {None: 0, "f32": 1, "f16": 2}


def make_opts(k=None, tol=None, prec="f64", rule="pivot_rel", k_max=0, nb=0, no_pivot=False,
              profile=False, gram=False, round_to=None, cholqr=False):
    """round_to: None, "f32" or "f16" -- the simulated single / half precision
    of the paper's Section 3 (ID_FLAG_ROUND_F32 / ID_FLAG_ROUND_F16)."""
    if prec not in PREC:
        raise ValueError(f"prec must be one of {sorted(PREC)}")
    if rule not in RULE:
        raise ValueError(f"rule must be one of {sorted(RULE)}")
    if round_to not in ROUND:
        raise ValueError('round_to must be None, "f32" or "f16"')
    if k is None and tol is None:
        raise ValueError("give k (fixed rank) or tol (adaptive rank)")
    o = _lib.IdOpts()
    o.prec = PREC[prec]
    o.rank_rule = RULE[rule]
    o.k_fixed = int(k) if k is not None else 0
    o.rel_tol = float(tol) if tol is not None else 0.0
    o.k_max = int(k_max)
    o.nb = int(nb)
    o.flags = ((C["ID_FLAG_NO_PIVOT"] if no_pivot else 0) | (C["ID_FLAG_PROFILE"] if profile else 0)
               | (C["ID_FLAG_GRAM"] if gram else 0)
               | (C["ID_FLAG_CHOLQR"] if cholqr else 0)
               | (C["ID_FLAG_ROUND_F32"] if round_to == "f32" else 0)
               | (C["ID_FLAG_ROUND_F16"] if round_to == "f16" else 0))
    if k is not None and int(k) == 0:
        o.k_max = 0
    return o


def workspace_size(m: int, n: int, dtype: torch.dtype, opts) -> int:
    return int(_lib.load().id_workspace_size(m, n, DTYPE[dtype], ctypes.byref(opts)))


def kcap_of(m: int, n: int, opts) -> int:
    kc = min(m, n)
    if opts.k_max > 0:
        kc = min(kc, opts.k_max)
    if opts.k_fixed > 0:
        kc = min(kc, opts.k_fixed)
    return kc


@dataclass
class FactorResult:
    perm: torch.Tensor  # (n,) int32
    R: torch.Tensor     # (k, n) float64, column-major view
    k: int
    info: int


def factor(A: torch.Tensor, k=None, tol=None, prec="f64", rule="pivot_rel", k_max=0, nb=0,
           no_pivot=False, work: torch.Tensor | None = None, R_buf: torch.Tensor | None = None,
           perm_buf: torch.Tensor | None = None, profile: bool = False,
           gram: bool = False, round_to=None, cholqr: bool = False) -> FactorResult:
    """Rank-k column-pivoted QR (id_factor).  k=0 gives k = 0.  gram=True takes
    the tall-skinny front end (pivots and R from the FP64 Gram matrix);
    cholqr=True the one through a shifted CholeskyQR3 R factor (full
    numerical column rank required; info ID_INFO_CHOLQR_BREAKDOWN otherwise)."""
    lib = _lib.load()
    A, lda = colmajor(A)
    m, n = A.shape
    if k is not None and int(k) == 0:
        return FactorResult(torch.arange(n, dtype=torch.int32, device=A.device),
                            empty_colmajor(0, n, device=A.device), 0, 0)
    o = make_opts(k, tol, prec, rule, k_max, nb, no_pivot, profile, gram, round_to, cholqr)
    ws = workspace_size(m, n, A.dtype, o)
    if ws == 0:
        raise ValueError("invalid factorization arguments")
    if work is None or work.numel() < ws:
        work = torch.empty(ws, dtype=torch.uint8, device=A.device)
    kc = kcap_of(m, n, o)
    if R_buf is None:
        R_buf = empty_colmajor(max(kc, 1), n, device=A.device)
    if perm_buf is None:
        perm_buf = torch.empty(n, dtype=torch.int32, device=A.device)
    ldr = max(R_buf.stride(1), 1) if n > 1 else max(kc, 1)
    k_out = ctypes.c_int64(0)
    info = ctypes.c_int32(0)
    with torch.cuda.device(A.device):
        rc = lib.id_factor(A.data_ptr(), DTYPE[A.dtype], m, n, lda, ctypes.byref(o),
                           work.data_ptr(), work.numel(), perm_buf.data_ptr(), R_buf.data_ptr(),
                           ldr, ctypes.byref(k_out), ctypes.byref(info), _stream(A.device))
    _lib.check(rc, "id_factor")
    kk = int(k_out.value)
    return FactorResult(perm_buf, R_buf[:kk], kk, int(info.value))


def factor_noalloc(A: torch.Tensor, k=None, tol=None, prec="f64", rule="pivot_rel", k_max=0,
                   nb=0, no_pivot=False, R_buf: torch.Tensor | None = None,
                   perm_buf: torch.Tensor | None = None) -> FactorResult:
    """id_factor_noalloc: the factorization of factor() in the library's static
    scratch (no workspace argument).  The library allocates nothing; this
    wrapper allocates R and perm unless the caller passes them."""
    lib = _lib.load()
    A, lda = colmajor(A)
    m, n = A.shape
    if k is not None and int(k) == 0:
        return FactorResult(torch.arange(n, dtype=torch.int32, device=A.device),
                            empty_colmajor(0, n, device=A.device), 0, 0)
    o = make_opts(k, tol, prec, rule, k_max, nb, no_pivot, False, False)
    kc = kcap_of(m, n, o)
    if R_buf is None:
        R_buf = empty_colmajor(max(kc, 1), n, device=A.device)
    if perm_buf is None:
        perm_buf = torch.empty(n, dtype=torch.int32, device=A.device)
    ldr = max(R_buf.stride(1), 1) if n > 1 else max(kc, 1)
    k_out = ctypes.c_int64(0)
    info = ctypes.c_int32(0)
    with torch.cuda.device(A.device):
        rc = lib.id_factor_noalloc(A.data_ptr(), DTYPE[A.dtype], m, n, lda, ctypes.byref(o),
                                   perm_buf.data_ptr(), R_buf.data_ptr(), ldr, ctypes.byref(k_out),
                                   ctypes.byref(info), _stream(A.device))
    _lib.check(rc, "id_factor_noalloc")
    kk = int(k_out.value)
    return FactorResult(perm_buf, R_buf[:kk], kk, int(info.value))


def solve_T(R: torch.Tensor, k: int, n: int, T_buf: torch.Tensor | None = None,
            check: bool = True):
    """T = R11^{-1} R12 (id_solve_T).  Returns (T, info) with info a device int32
    tensor; with check=True the call waits for info and raises when singular."""
    lib = _lib.load()
    dev = R.device
    ldr = R.stride(1) if R.dim() == 2 and n > 1 else max(k, 1)
    if T_buf is None:
        T_buf = empty_colmajor(k, n - k, device=dev)
    ldt = T_buf.stride(1) if (n - k) > 1 else max(k, 1)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    with torch.cuda.device(dev):
        rc = lib.id_solve_T(R.data_ptr(), ldr, k, n, T_buf.data_ptr(), max(ldt, 1),
                            info.data_ptr(), _stream(dev))
    _lib.check(rc, "id_solve_T")
    if check:
        code = int(info.item())
        if code == C["ID_INFO_SINGULAR"]:
            raise _lib.MpidError(code, "id_solve_T")
    return T_buf[:k], info


def reconstruct(A: torch.Tensor, perm: torch.Tensor, k: int, T: torch.Tensor,
                residual: bool = False) -> torch.Tensor:
    """Y = A(:, J) P in float64 (or A - Y with residual=True), column-major."""
    lib = _lib.load()
    A, lda = colmajor(A)
    m, n = A.shape
    Y = empty_colmajor(m, n, device=A.device)
    Tc = T if (T.numel() == 0 or T.stride(0) == 1) else T.t().contiguous().t()
    ldt = Tc.stride(1) if (n - k) > 1 else max(k, 1)
    with torch.cuda.device(A.device):
        rc = lib.id_reconstruct(A.data_ptr(), DTYPE[A.dtype], m, n, lda, perm.data_ptr(), k,
                                Tc.data_ptr() if Tc.numel() else None, max(ldt, 1), Y.data_ptr(),
                                Y.stride(1) if n > 1 else max(m, 1), int(residual),
                                _stream(A.device))
    _lib.check(rc, "id_reconstruct")
    return Y


def backward(A: torch.Tensor, perm: torch.Tensor, k: int, T: torch.Tensor, gT=None, gY=None,
             R11: torch.Tensor | None = None):
    """Adjoint with the skeleton fixed (id_backward): returns gA (float64, m x n).
    R11: optional k x k R factor of A(:, perm[:k]) (e.g. the first k columns
    of an FP64 factor()'s R) -- saves the QR of the skeleton."""
    lib = _lib.load()
    A, lda = colmajor(A)
    m, n = A.shape
    dev = A.device
    gA = empty_colmajor(m, n, device=dev)
    Tc = T if (T.numel() == 0 or T.stride(0) == 1) else T.t().contiguous().t()
    ldt = max(Tc.stride(1) if (n - k) > 1 else k, 1)
    gTc = None
    if gT is not None:
        gTc = gT.to(torch.float64)
        gTc = gTc if (gTc.numel() == 0 or gTc.stride(0) == 1) else gTc.t().contiguous().t()
    gYc = None
    if gY is not None:
        gYc, _ = colmajor(gY.to(torch.float64))
    Rc = None
    if R11 is not None and k > 0:
        if tuple(R11.shape) != (k, k) or R11.dtype != torch.float64:
            raise ValueError("R11 must be a k x k float64 matrix")
        Rc = R11 if R11.stride(0) == 1 else R11.t().contiguous().t()
    ws = int(lib.id_backward_workspace_size(m, n, k))
    work = torch.empty(max(ws, 1), dtype=torch.uint8, device=dev)
    info = ctypes.c_int32(0)
    with torch.cuda.device(dev):
        rc = lib.id_backward(
            A.data_ptr(), DTYPE[A.dtype], m, n, lda, perm.data_ptr(), k,
            Tc.data_ptr() if Tc.numel() else None, ldt,
            Rc.data_ptr() if Rc is not None else None,
            max(Rc.stride(1), k) if Rc is not None and k > 1 else max(k, 1),
            gTc.data_ptr() if gTc is not None and gTc.numel() else None,
            max(gTc.stride(1) if (gTc is not None and (n - k) > 1) else k, 1),
            gYc.data_ptr() if gYc is not None else None,
            gYc.stride(1) if gYc is not None and n > 1 else max(m, 1),
            gA.data_ptr(), gA.stride(1) if n > 1 else max(m, 1), work.data_ptr(), work.numel(),
            ctypes.byref(info), _stream(dev))
    _lib.check(rc, "id_backward")
    if info.value == C["ID_INFO_SINGULAR"]:
        raise _lib.MpidError(info.value, "id_backward")
    return gA


def last_profile() -> dict:
    """Per-kernel event timings of this thread's last factor(..., profile=True)."""
    p = _lib.IdProfile()
    _lib.check(_lib.load().id_last_profile(ctypes.byref(p)), "id_last_profile")
    return p.as_dict()


@dataclass
class ColumnIDResult:
    J: torch.Tensor     # (k,) int64 skeleton
    T: torch.Tensor     # (k, n-k) float64
    perm: torch.Tensor  # (n,) int32
    k: int
    R: torch.Tensor     # (k, n) float64
    info: int = 0       # id_factor's info (e.g. ID_INFO_GRAM_LIMIT)


def round_(X: torch.Tensor, mode: str) -> torch.Tensor:
    """id_round: X (float64, column-major view) rounded in place to binary32
    ("f32") or binary16 ("f16") values."""
    if X.numel() == 0:
        return X
    rows, cols = X.shape
    ld = X.stride(1) if cols > 1 else max(rows, 1)
    if X.dtype != torch.float64 or X.stride(0) != 1:
        raise ValueError("id_round takes a float64 column-major matrix")
    with torch.cuda.device(X.device):
        _lib.check(_lib.load().id_round(X.data_ptr(), rows, cols, ld, ROUND[mode],
                                        _stream(X.device)), "id_round")
    return X


def column_id(A: torch.Tensor, k=None, tol=None, prec="f64", rule="pivot_rel", k_max=0, nb=0,
              gram=False, round_to=None, cholqr=False):
    """Algorithm 1 (prec="f64") or Algorithm 2's mixed variant end to end
    (gram=True: the Gram-matrix front end for tall inputs; round_to="f32" /
    "f16": the simulated single / half precision ID, T rounded too)."""
    fr = factor(A, k=k, tol=tol, prec=prec, rule=rule, k_max=k_max, nb=nb, gram=gram,
                round_to=round_to, cholqr=cholqr)
    n = A.shape[1]
    T, _ = solve_T(fr.R, fr.k, n)
    if round_to is not None:
        round_(T, round_to)
    return ColumnIDResult(fr.perm[:fr.k].long(), T, fr.perm, fr.k, fr.R, fr.info)


class ColumnID(torch.autograd.Function):
    """(T, Y) = ID of A with Y = A(:, J) P; the backward holds J fixed and uses
    id_backward.  k, the permutation and R are exposed as non-differentiable
    attributes of the context via ``last``."""

    last = None

    @staticmethod
    def forward(ctx, A, k=None, tol=None, prec="f64", rule="pivot_rel"):
        res = column_id(A.detach(), k=k, tol=tol, prec=prec, rule=rule)
        Y = reconstruct(A.detach(), res.perm, res.k, res.T)
        # an FP64 forward's R11 is the skeleton's R factor: the backward reuses it
        R11 = res.R[:, :res.k] if prec == "f64" else res.R.new_empty(0)
        ctx.save_for_backward(A.detach(), res.perm, res.T, R11)
        ctx.k = res.k
        ColumnID.last = res
        return res.T, Y

    @staticmethod
    def backward(ctx, gT, gY):
        A, perm, T, R11 = ctx.saved_tensors
        gA = backward(A, perm, ctx.k, T, gT=gT, gY=gY, R11=R11 if R11.numel() else None)
        return gA.to(A.dtype), None, None, None, None


def sketch(A: torch.Tensor, Omega: torch.Tensor) -> torch.Tensor:
    """Y = Omega A (id_sketch): Omega l x m float64, A m x n; Y l x n float64,
    column-major."""
    lib = _lib.load()
    A, lda = colmajor(A)
    m, n = A.shape
    if Omega.dim() != 2 or Omega.shape[1] != m or Omega.dtype != torch.float64:
        raise ValueError("Omega must be an l x m float64 matrix")
    if Omega.device != A.device:
        raise ValueError("Omega and A must be on the same device")
    l = Omega.shape[0]
    # row-major Omega: unit stride along the rows of A
    Om = Omega if (m <= 1 or Omega.stride(1) == 1) else Omega.contiguous()
    ldo = max(Om.stride(0) if l > 1 else m, m, 1)
    Y = empty_colmajor(l, n, device=A.device)
    ws = int(lib.id_sketch_workspace_size(l, m, n))
    work = torch.empty(max(ws, 8), dtype=torch.uint8, device=A.device)
    with torch.cuda.device(A.device):
        rc = lib.id_sketch(A.data_ptr(), DTYPE[A.dtype], m, n, lda, Om.data_ptr(), l, ldo,
                           Y.data_ptr(), Y.stride(1) if n > 1 else max(l, 1), work.data_ptr(),
                           work.numel(), _stream(A.device))
    _lib.check(rc, "id_sketch")
    return Y


@dataclass
class SketchIDResult(ColumnIDResult):
    Y: torch.Tensor = None  # (l, n) float64 sketch Omega A


def sketch_id(A: torch.Tensor, Omega: torch.Tensor, k=None, tol=None, rule="pivot_rel",
              k_max=0) -> SketchIDResult:
    """Randomized column ID: Y = Omega A (id_sketch), then the FP64
    column-pivoted factorization of Y (id_factor) and T from Y's R
    (id_solve_T); A ~ A[:, J] T.  Rank rules act on Y's residual norms."""
    Y = sketch(A, Omega)
    res = column_id(Y, k=k, tol=tol, prec="f64", rule=rule, k_max=k_max)
    return SketchIDResult(res.J, res.T, res.perm, res.k, res.R, res.info, Y=Y)
