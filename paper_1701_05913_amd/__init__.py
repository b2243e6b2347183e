"""Python binding of libkrylov.so, the gfx950 preconditioned Krylov solver.

The functions below carry the names of the C ABI in include/krylov.h and do
argument marshalling only: torch CUDA tensors are passed as device
pointers, numpy arrays as host pointers, and every computation runs in the
library's HIP kernels.  There is no fallback: importing this package fails
when the library has not been built, and every call raises KrylovError
when the library reports an error.

Build with `python paper_1701_05913_amd/build.py` (or
`__graft_entry__.build()`).

torch ships its own HIP runtime; the binding imports torch before it
loads the library, so that the library binds to the runtime already in
the process and both share one GPU context.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBRARY = os.path.join(_HERE, "libkrylov.so")

# status codes and enumerations (include/krylov.h)
KRY_OK, KRY_NOT_CONVERGED = 0, 1
KRY_ERR_ARG, KRY_ERR_DIM, KRY_ERR_ALLOC, KRY_ERR_ZERO_PIVOT = -1, -2, -3, -4
KRY_ERR_BREAKDOWN, KRY_ERR_HIP, KRY_ERR_UNSUPPORTED, KRY_ERR_STALL = -5, -6, -7, -8
KRY_HOST, KRY_DEVICE = 0, 1
KRY_F64 = 0
KRY_GMRES, KRY_FGMRES, KRY_BICGSTAB, KRY_CG = 0, 1, 2, 3
KRY_PC_NONE, KRY_PC_ILU0, KRY_PC_BILU0, KRY_PC_CPR, KRY_PC_CUSTOM = 0, 1, 1, 2, 3
KRY_PC_BILU0_LEARNED, KRY_PC_CPR_LEARNED, KRY_PC_RAS, KRY_PC_AMG = 4, 5, 6, 7
KRY_PREC_F64, KRY_PREC_F32, KRY_PREC_BF16_FACTORS = 0, 1, 2
KRY_CPR_PF, KRY_CPR_FP, KRY_CPR_FPF, KRY_CPR_FFPF = 0, 1, 2, 3
KRY_CPR_P_ILU0, KRY_CPR_P_AMG = 0, 1
KRY_CPR_F_BILU0, KRY_CPR_F_RAS = 0, 1
KRY_SWEEP_AUTO, KRY_SWEEP_LEVELS, KRY_SWEEP_GRID = 0, 1, 2
KRY_ORTHO_AUTO, KRY_ORTHO_CGS2 = 0, 1


class KrylovError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


if not os.path.exists(LIBRARY):
    raise ImportError(f"{LIBRARY} is not built; run `python paper_1701_05913_amd/build.py`")

# one HIP runtime per process: torch's, loaded before the library (the
# library's own dependency then resolves to it)
import torch  # noqa: E402,F401

_lib = C.CDLL(LIBRARY)

P, D, I32, I64 = C.c_void_p, C.c_double, C.c_int32, C.c_int64
_SIGS = {
    "MapCreate": (P, [I64, I64]), "MapCreateLocal": (P, [I64]),
    "MapDestroy": (None, [P]), "MapGetNlocal": (I64, [P]),
    "VecCreate": (P, [P, C.c_int]), "VecWrap": (P, [P, P, C.c_int]),
    "VecDestroy": (None, [C.POINTER(P)]), "VecGetData": (P, [P]),
    "VecAddEntry": (C.c_int, [P, I64, D]), "VecGetEntry": (D, [P, I64]),
    "VecSetValue": (C.c_int, [P, D]), "VecAXPBY": (C.c_int, [D, P, D, P]),
    "VecAXPBYZ": (C.c_int, [D, P, D, P, P]), "VecDot": (D, [P, P]),
    "VecNorm2": (D, [P]),
    "MatCreateCSR": (P, [P, I32, P, P, P, C.c_int]),
    "MatCreateBSR": (P, [P, I32, I32, P, P, P, C.c_int]),
    "MatDestroy": (None, [C.POINTER(P)]), "MatVecMXY": (C.c_int, [P, P, P]),
    "MatUpdateValues": (C.c_int, [P, P, C.c_int]),
    "MatVecAMXPBY": (C.c_int, [D, P, P, D, P]), "MatGetNnzBlocks": (I64, [P]),
    "MatGetGrid": (C.c_int, [P, C.POINTER(I32), C.POINTER(I32), C.POINTER(I32)]),
    "SolverCreate": (P, [C.c_int, C.c_int, P]),
    "SolverDestroy": (C.c_int, [C.POINTER(P)]),
    "SolverSetMat": (C.c_int, [P, P]), "SolverAssemble": (C.c_int, [P]),
    "SolverSolve": (C.c_int, [P, P, P]), "SolverPCApply": (C.c_int, [P, P, P]),
    "SolverSetDefaultMaxit": (None, [I64]), "SolverSetDefaultRtol": (None, [D]),
    "SolverSetDefaultAtol": (None, [D]), "SolverSetDefaultBtol": (None, [D]),
    "SolverSetDefaultRestart": (None, [I64]), "SolverSetDefaultAugk": (None, [I64]),
    "SolverSetMaxit": (C.c_int, [P, I64]), "SolverSetRtol": (C.c_int, [P, D]),
    "SolverSetAtol": (C.c_int, [P, D]), "SolverSetBtol": (C.c_int, [P, D]),
    "SolverSetRestart": (C.c_int, [P, I64]), "SolverSetAugk": (C.c_int, [P, I64]),
    "SolverSetPrecision": (C.c_int, [P, C.c_int]),
    "SolverSetCPR": (C.c_int, [P, C.c_int, C.c_int]),
    "SolverSetRAS": (C.c_int, [P, C.c_int, C.c_int]),
    "SolverSetRASBoxes": (C.c_int, [P, C.c_int, C.c_int, C.c_int, C.c_int]),
    "SolverSetCPRPressure": (C.c_int, [P, C.c_int]),
    "SolverSetCPRFull": (C.c_int, [P, C.c_int]),
    "SolverSetAMG": (C.c_int, [P, C.c_int, C.c_int, C.c_int]),
    "SolverGetAMGLevels": (C.c_int, [P]),
    "SolverGetAMGLevel": (C.c_int, [P, C.c_int] + [C.POINTER(I32)] * 4 + [P] * 7),
    "SolverSetSweepLayout": (C.c_int, [P, C.c_int]),
    "SolverSetOrthog": (C.c_int, [P, C.c_int]),
    "SolverSetStream": (C.c_int, [P, P]),
    "SolverGetResidual": (D, [P]), "SolverGetIters": (C.c_int, [P]),
    "SolverGetTimes": (C.c_int, [P, C.POINTER(D), C.POINTER(D)]),
    "SolverGetHistory": (C.c_int, [P, P, C.c_int]),
    "VecDotNoAlloc": (C.c_int, [P, P, P]),
    "SolverGetKrylovBasis": (C.c_int, [P, C.c_int, C.c_int, P, C.c_int]),
    "SolverSetPC": (C.c_int, [P, P, P, P, P]),
    "KernelTimingEnable": (C.c_int, [C.c_int]), "KernelTimingReset": (C.c_int, []),
    "KernelTimingSelect": (C.c_int, [C.c_char_p]), "KernelTimingSample": (C.c_int, [C.c_int]),
    "KernelTimingQuery": (C.c_int, [C.c_char_p, C.POINTER(I64), C.POINTER(D)]),
    "KrylovSetStream": (C.c_int, [P]), "LastError": (C.c_char_p, []),
    "SolverSetLearned": (C.c_int, [P, C.c_char_p, P]),
    "SolverSetLearnedParams": (C.c_int, [P, P, P, C.c_int]),
    "SolverGetLearnedStats": (C.c_int, [P, C.POINTER(I64), C.POINTER(I64)]),
    "LearnedCreate": (P, [C.c_int, C.c_int, C.c_int, C.c_int]),
    "LearnedDestroy": (C.c_int, [C.POINTER(P)]), "LearnedNumParams": (C.c_int, []),
    "LearnedSetStream": (C.c_int, [P, P]),
    "LearnedSetParams": (C.c_int, [P, P, C.c_int]), "LearnedGetParams": (C.c_int, [P, P]),
    "LearnedForward": (C.c_int, [P, P, P]),
    "LearnedLossGrad": (C.c_int, [P, P, P, C.POINTER(C.c_float), P]),
    "LearnedAdamStep": (C.c_int, [P, C.c_float, C.c_float, C.c_float, C.c_float]),
    "LearnedSave": (C.c_int, [P, C.c_char_p]), "LearnedLoad": (C.c_int, [P, C.c_char_p]),
    "LearnedMakePair": (C.c_int, [I64, P, P, P, P, P, C.POINTER(D)]),
    "LearnedBackward": (C.c_int, [P, P, P]),
    "LearnedResidualGrad": (C.c_int, [P, P, P, P, P, P, C.POINTER(D)]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def LastError() -> str:
    return _lib.LastError().decode(errors="replace")


def _check(rc):
    if rc is not None and rc < 0:
        raise KrylovError(rc, LastError())
    return rc


def _handle(h, what):
    if not h:
        raise KrylovError(None, f"{what}: {LastError()}")
    return h


def _ptr(a, dtype):
    """(pointer, where) of a torch tensor or numpy array with the given
    element type (np.int32 / np.float64)."""
    if hasattr(a, "data_ptr"):                      # torch tensor
        import torch
        tdt = {np.int32: torch.int32, np.float64: torch.float64}[dtype]
        if a.dtype != tdt:
            raise TypeError(f"expected {tdt}, got {a.dtype}")
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return C.c_void_p(a.data_ptr()), (KRY_DEVICE if a.is_cuda else KRY_HOST)
    a = np.asarray(a)
    if a.dtype != dtype or not a.flags["C_CONTIGUOUS"]:
        raise TypeError(f"expected a contiguous {np.dtype(dtype)} array")
    return a.ctypes.data_as(C.c_void_p), KRY_HOST


def _dptr(t):
    """Device pointer of a CUDA float64 tensor."""
    if not (hasattr(t, "is_cuda") and t.is_cuda):
        raise TypeError("expected a CUDA tensor")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return C.c_void_p(t.data_ptr())


# ---- MAP -----------------------------------------------------------------
def MapCreate(ilower, iupper):
    return _handle(_lib.MapCreate(ilower, iupper), "MapCreate")


def MapCreateLocal(nlocal):
    return _handle(_lib.MapCreateLocal(nlocal), "MapCreateLocal")


def MapDestroy(m):
    _lib.MapDestroy(m)


def MapGetNlocal(m):
    return _lib.MapGetNlocal(m)


# ---- VEC -----------------------------------------------------------------
def VecCreate(m, dtype=KRY_F64):
    return _handle(_lib.VecCreate(m, dtype), "VecCreate")


def VecWrap(m, tensor, dtype=KRY_F64):
    """Borrow a CUDA float64 tensor (the caller keeps it alive)."""
    import torch
    if tensor.dtype != torch.float64:
        raise TypeError("VecWrap needs a float64 tensor")
    return _handle(_lib.VecWrap(m, _dptr(tensor), dtype), "VecWrap")


def VecDestroy(v):
    h = C.c_void_p(v)
    _lib.VecDestroy(C.byref(h))


def VecGetData(v):
    return _lib.VecGetData(v)


def VecAddEntry(v, idx, value):
    return _check(_lib.VecAddEntry(v, idx, value))


def VecGetEntry(v, idx):
    return _lib.VecGetEntry(v, idx)


def VecSetValue(v, value):
    return _check(_lib.VecSetValue(v, value))


def VecAXPBY(a, x, b, y):
    return _check(_lib.VecAXPBY(a, x, b, y))


def VecAXPBYZ(a, x, b, y, z):
    return _check(_lib.VecAXPBYZ(a, x, b, y, z))


def VecDot(x, y):
    return _lib.VecDot(x, y)


def VecNorm2(x):
    return _lib.VecNorm2(x)


def VecDotNoAlloc(x, y, result):
    """<x, y> into `result`, a CUDA float64 tensor (its first element),
    asynchronously on the library stream, without allocating."""
    return _check(_lib.VecDotNoAlloc(x, y, _dptr(result)))


# ---- MAT -----------------------------------------------------------------
def MatCreateCSR(m, n, rowptr, col, val):
    rp, w1 = _ptr(rowptr, np.int32)
    cp, w2 = _ptr(col, np.int32)
    vp, w3 = _ptr(val, np.float64)
    if not (w1 == w2 == w3):
        raise ValueError("rowptr, col and val must all be host or all device")
    return _handle(_lib.MatCreateCSR(m, n, rp, cp, vp, w1), "MatCreateCSR")


def MatCreateBSR(m, nb, bs, browptr, bcol, bval):
    rp, w1 = _ptr(browptr, np.int32)
    cp, w2 = _ptr(bcol, np.int32)
    vp, w3 = _ptr(bval, np.float64)
    if not (w1 == w2 == w3):
        raise ValueError("browptr, bcol and bval must all be host or all device")
    return _handle(_lib.MatCreateBSR(m, nb, bs, rp, cp, vp, w1), "MatCreateBSR")


def MatDestroy(a):
    h = C.c_void_p(a)
    _lib.MatDestroy(C.byref(h))


def MatUpdateValues(a, val):
    vp, w = _ptr(val, np.float64)
    return _check(_lib.MatUpdateValues(a, vp, w))


def MatVecMXY(a, x, y):
    return _check(_lib.MatVecMXY(a, x, y))


def MatVecAMXPBY(alpha, a, x, beta, y):
    return _check(_lib.MatVecAMXPBY(alpha, a, x, beta, y))


def MatGetNnzBlocks(a):
    return _lib.MatGetNnzBlocks(a)


def MatGetGrid(a):
    """(nx, ny, nz) of the recognised 7-point grid, or None."""
    nx, ny, nz = C.c_int32(0), C.c_int32(0), C.c_int32(0)
    rc = _lib.MatGetGrid(a, C.byref(nx), C.byref(ny), C.byref(nz))
    return (nx.value, ny.value, nz.value) if rc == 0 else None


# ---- SOLVER --------------------------------------------------------------
def SolverCreate(solver_type, pc_type, m):
    return _handle(_lib.SolverCreate(solver_type, pc_type, m), "SolverCreate")


def SolverDestroy(s):
    h = C.c_void_p(s)
    return _check(_lib.SolverDestroy(C.byref(h)))


def SolverSetMat(s, a):
    return _check(_lib.SolverSetMat(s, a))


def SolverAssemble(s):
    return _check(_lib.SolverAssemble(s))


def SolverSolve(s, b, x):
    return _check(_lib.SolverSolve(s, b, x))


def SolverPCApply(s, v, z):
    return _check(_lib.SolverPCApply(s, v, z))


def SolverSetDefaultMaxit(it): _lib.SolverSetDefaultMaxit(it)
def SolverSetDefaultRtol(t): _lib.SolverSetDefaultRtol(t)
def SolverSetDefaultAtol(t): _lib.SolverSetDefaultAtol(t)
def SolverSetDefaultBtol(t): _lib.SolverSetDefaultBtol(t)
def SolverSetDefaultRestart(m): _lib.SolverSetDefaultRestart(m)
def SolverSetDefaultAugk(k): _lib.SolverSetDefaultAugk(k)
def SolverSetMaxit(s, it): return _check(_lib.SolverSetMaxit(s, it))
def SolverSetRtol(s, t): return _check(_lib.SolverSetRtol(s, t))
def SolverSetAtol(s, t): return _check(_lib.SolverSetAtol(s, t))
def SolverSetBtol(s, t): return _check(_lib.SolverSetBtol(s, t))
def SolverSetRestart(s, m): return _check(_lib.SolverSetRestart(s, m))
def SolverSetAugk(s, k): return _check(_lib.SolverSetAugk(s, k))
def SolverSetPrecision(s, p): return _check(_lib.SolverSetPrecision(s, p))
def SolverSetCPR(s, variant, p_sweeps): return _check(_lib.SolverSetCPR(s, variant, p_sweeps))
def SolverSetRAS(s, nsub, overlap): return _check(_lib.SolverSetRAS(s, nsub, overlap))
def SolverSetRASBoxes(s, px, py, pz, overlap): return _check(_lib.SolverSetRASBoxes(s, px, py, pz, overlap))
def SolverSetCPRPressure(s, psolver): return _check(_lib.SolverSetCPRPressure(s, psolver))
def SolverSetCPRFull(s, fsolver): return _check(_lib.SolverSetCPRFull(s, fsolver))
def SolverSetAMG(s, max_levels, num_sweeps, gs_chunk):
    return _check(_lib.SolverSetAMG(s, max_levels, num_sweeps, gs_chunk))
def SolverGetAMGLevels(s): return _check(_lib.SolverGetAMGLevels(s))


def SolverGetAMGLevel(s, level):
    """dict(n, nc, A=(rowptr, col, val), cf, P=(rowptr, col, val)); cf and P
    are None on the coarsest level."""
    n, nnz, nc, pnnz = (C.c_int32(0) for _ in range(4))
    null = [None] * 7
    _check(_lib.SolverGetAMGLevel(s, level, C.byref(n), C.byref(nnz), C.byref(nc), C.byref(pnnz),
                                  *null))
    n, nnz, nc, pnnz = n.value, nnz.value, nc.value, pnnz.value
    rp = np.zeros(n + 1, np.int32)
    col = np.zeros(max(nnz, 1), np.int32)
    val = np.zeros(max(nnz, 1))
    cf = np.zeros(max(n, 1), np.int32)
    prp = np.zeros(n + 1, np.int32)
    pcol = np.zeros(max(pnnz, 1), np.int32)
    pval = np.zeros(max(pnnz, 1))
    ptr = [a.ctypes.data_as(C.c_void_p) for a in (rp, col, val, cf, prp, pcol, pval)]
    _check(_lib.SolverGetAMGLevel(s, level, None, None, None, None, *ptr))
    coarse = nc == 0
    return dict(n=n, nc=nc, A=(rp, col[:nnz], val[:nnz]), cf=None if coarse else cf[:n],
                P=None if coarse else (prp, pcol[:pnnz], pval[:pnnz]))
def SolverSetSweepLayout(s, layout): return _check(_lib.SolverSetSweepLayout(s, layout))
def SolverSetOrthog(s, kind): return _check(_lib.SolverSetOrthog(s, kind))


def SolverSetStream(s, stream):
    """stream: a torch.cuda.Stream, a raw hipStream_t integer, or None."""
    raw = getattr(stream, "cuda_stream", stream)
    return _check(_lib.SolverSetStream(s, C.c_void_p(raw or 0)))


def SolverGetResidual(s):
    return _lib.SolverGetResidual(s)


def SolverGetIters(s):
    return _lib.SolverGetIters(s)


def SolverGetTimes(s):
    a, b = C.c_double(0), C.c_double(0)
    _check(_lib.SolverGetTimes(s, C.byref(a), C.byref(b)))
    return a.value, b.value


def SolverGetHistory(s, cap=100000):
    buf = np.zeros(cap)
    k = _check(_lib.SolverGetHistory(s, buf.ctypes.data_as(C.c_void_p), cap))
    return buf[:k].copy()


def SolverGetKrylovBasis(s, first, ncols, n, out=None):
    """Columns [first, first + ncols) of the last cycle's basis: into `out`
    (a contiguous CUDA float64 tensor of ncols * n values) when given, else
    as a host array of shape (ncols, n)."""
    if out is not None:
        _check(_lib.SolverGetKrylovBasis(s, first, ncols, _dptr(out), KRY_DEVICE))
        return out
    buf = np.zeros((ncols, n))
    _check(_lib.SolverGetKrylovBasis(s, first, ncols, buf.ctypes.data_as(C.c_void_p), KRY_HOST))
    return buf


PC_SETUP = C.CFUNCTYPE(C.c_int, C.c_void_p, C.c_void_p)
PC_SOLVE = C.CFUNCTYPE(C.c_int, C.c_void_p, C.c_void_p, C.c_void_p)
PC_DESTROY = C.CFUNCTYPE(None, C.c_void_p)


def SolverSetPC(s, setup, solve, destroy, data=None):
    """setup/solve/destroy: PC_SETUP / PC_SOLVE / PC_DESTROY instances (the
    caller keeps them alive as long as the solver)."""
    return _check(_lib.SolverSetPC(s, setup, solve, destroy, data))


# ---- learned stage ---------------------------------------------------------------
def _fptr(a):
    """(pointer, where) of a float32 torch tensor or numpy array."""
    if hasattr(a, "data_ptr"):
        import torch
        if a.dtype != torch.float32 or not a.is_contiguous():
            raise TypeError("expected a contiguous float32 tensor")
        return C.c_void_p(a.data_ptr()), (KRY_DEVICE if a.is_cuda else KRY_HOST)
    a = np.asarray(a)
    if a.dtype != np.float32 or not a.flags["C_CONTIGUOUS"]:
        raise TypeError("expected a contiguous float32 array")
    return a.ctypes.data_as(C.c_void_p), KRY_HOST


def _fdptr(t):
    p, where = _fptr(t)
    if where != KRY_DEVICE:
        raise TypeError("expected a CUDA float32 tensor")
    return p


def SolverSetLearned(s, weights_path, logk_dev):
    return _check(_lib.SolverSetLearned(s, os.fsencode(weights_path), _fdptr(logk_dev)))


def SolverSetLearnedParams(s, params, logk):
    pp, pw = _fptr(params)
    if pw != KRY_HOST:
        raise TypeError("parameters must be a host float32 array")
    lp, lw = _fptr(logk)
    return _check(_lib.SolverSetLearnedParams(s, pp, lp, lw))


def SolverGetLearnedStats(s):
    a, f = C.c_int64(0), C.c_int64(0)
    _check(_lib.SolverGetLearnedStats(s, C.byref(a), C.byref(f)))
    return a.value, f.value


def LearnedMakePair(cells, r1, d, logk, inp, target):
    """Returns s; r1, d: CUDA float64 tensors; logk, inp, target: CUDA float32."""
    sv = C.c_double(0)
    _check(_lib.LearnedMakePair(cells, _dptr(r1), _dptr(d), _fdptr(logk), _fdptr(inp),
                                _fdptr(target), C.byref(sv)))
    return sv.value


def LearnedCreate(nx, ny, nz, training=False):
    return _handle(_lib.LearnedCreate(nx, ny, nz, int(bool(training))), "LearnedCreate")


def LearnedDestroy(L):
    h = C.c_void_p(L)
    return _check(_lib.LearnedDestroy(C.byref(h)))


def LearnedNumParams():
    return _lib.LearnedNumParams()


def LearnedSetStream(L, stream):
    raw = getattr(stream, "cuda_stream", stream)
    return _check(_lib.LearnedSetStream(L, C.c_void_p(raw or 0)))


def LearnedSetParams(L, params):
    p, where = _fptr(params)
    return _check(_lib.LearnedSetParams(L, p, where))


def LearnedGetParams(L):
    out = np.zeros(LearnedNumParams(), dtype=np.float32)
    _check(_lib.LearnedGetParams(L, out.ctypes.data_as(C.c_void_p)))
    return out


def LearnedForward(L, inp, out):
    return _check(_lib.LearnedForward(L, _fdptr(inp), _fdptr(out)))


def LearnedLossGrad(L, inp, target, grad=None):
    loss = C.c_float(0)
    _check(_lib.LearnedLossGrad(L, _fdptr(inp), _fdptr(target), C.byref(loss),
                                _fdptr(grad) if grad is not None else None))
    return loss.value


def LearnedBackward(L, dout, grad=None):
    return _check(_lib.LearnedBackward(L, _fdptr(dout), _fdptr(grad) if grad is not None else None))


def LearnedResidualGrad(L, A, At, inp, out, dout):
    """Returns the residual loss; A, At: MAT handles."""
    lv = C.c_double(0)
    _check(_lib.LearnedResidualGrad(L, A, At, _fdptr(inp), _fdptr(out), _fdptr(dout), C.byref(lv)))
    return lv.value


def LearnedAdamStep(L, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    return _check(_lib.LearnedAdamStep(L, lr, beta1, beta2, eps))


def LearnedSave(L, path):
    return _check(_lib.LearnedSave(L, os.fsencode(path)))


def LearnedLoad(L, path):
    return _check(_lib.LearnedLoad(L, os.fsencode(path)))


# ---- timing and stream ---------------------------------------------------------
def KernelTimingEnable(on=True):
    return _check(_lib.KernelTimingEnable(int(bool(on))))


def KernelTimingSelect(names=None):
    """Time only the named kernel families (a comma-separated string or a
    list of names); None times every family."""
    if names is not None and not isinstance(names, str):
        names = ",".join(names)
    return _check(_lib.KernelTimingSelect(None if names is None else names.encode()))


def KernelTimingSample(every=1):
    """Bracket only the first of every `every` launches of each family."""
    return _check(_lib.KernelTimingSample(int(every)))


def KernelTimingReset():
    return _check(_lib.KernelTimingReset())


def KernelTimingQuery(name):
    n, ms = C.c_int64(0), C.c_double(0)
    _check(_lib.KernelTimingQuery(name.encode(), C.byref(n), C.byref(ms)))
    return n.value, ms.value


def KrylovSetStream(stream):
    raw = getattr(stream, "cuda_stream", stream)
    return _check(_lib.KrylovSetStream(C.c_void_p(raw or 0)))


def exported_symbols():
    """Names of every C-ABI function this binding declares."""
    return sorted(_SIGS)
