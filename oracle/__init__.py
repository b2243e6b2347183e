"""Python access to the FP64 CPU oracle (oracle.c) through ctypes.

TEST INFRASTRUCTURE ONLY: imported by the tests, by the package smoke check
and by the CPU-baseline leg of the benchmark.  The GPU library and its
Python binding never import this package, and this package never imports
them.

Systems are the dicts produced by `reservoir_inputs` (keys rowptr, col,
val, and bs for block systems).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

OK, NOT_CONVERGED, ERR_ARG, ERR_ZERO_PIVOT, ERR_BREAKDOWN = 0, 1, -1, -4, -5
PREC = {"f64": 0, "f32": 1, "bf16": 2}
PC_KIND = {"none": 0, "bilu0": 1, "ilu0": 1, "cpr_pf": 2, "cpr_fp": 3,
           "cpr_fpf": 5, "cpr_ffpf": 6, "amg": 8}


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (plain -O2, no fast-math, no FMA
    contraction)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
             "-fno-fast-math", "-Wall", "-Wno-unknown-pragmas", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_SO_OMP = os.path.join(_HERE, "liboracle_omp.so")


def build_omp(force: bool = True) -> str:
    """The same source with OpenMP on (parallel SpMV, dot products and the
    vector loops of GMRES; serial sweeps and factorization): the
    multi-threaded CPU timing leg, never a parity reference."""
    if force or not os.path.exists(_SO_OMP):
        tmp = _SO_OMP + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
             "-fno-fast-math", "-fopenmp", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO_OMP)
    return _SO_OMP


class using:
    """Context manager: route this module's calls through another compiled
    oracle library (e.g. load(build_omp(False)))."""

    def __init__(self, lib_):
        self.lib = lib_

    def __enter__(self):
        global _lib
        self.saved = _lib
        _lib = self.lib
        return self.lib

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


_lib = None


def load(path: str):
    """Open a compiled oracle library and declare its signatures."""
    L = C.CDLL(path)
    P, D, I = C.c_void_p, C.c_double, C.c_int
    L.or_bsr_spmv.argtypes = [I, I, P, P, P, P, P]
    L.or_bsr_amxpby.argtypes = [I, I, P, P, P, D, P, D, P]
    L.or_bilu0.argtypes = [I, I, P, P, P, P]
    L.or_bilu0.restype = I
    L.or_bilu0_solve.argtypes = [I, I, P, P, P, P, P]
    L.or_bilu0_solve_lower.argtypes = [I, I, P, P, P, P, P]
    L.or_bilu0_solve_upper.argtypes = [I, I, P, P, P, P, P]
    L.or_pc_create.argtypes = [I, I, I, P, P, P, I, I, C.POINTER(I)]
    L.or_pc_create.restype = P
    L.or_pc_create_learned.argtypes = [P, I, I, I, P, P, I]
    L.or_pc_create_ras.argtypes = [I, I, P, P, P, I, P, I, C.POINTER(I)]
    L.or_pc_create_ras.restype = P
    L.or_pc_create_ras_part.argtypes = [I, I, P, P, P, I, P, I, C.POINTER(I)]
    L.or_pc_create_ras_part.restype = P
    L.or_pc_create_ras_sets.argtypes = [I, I, P, P, P, I, P, P, P, C.POINTER(I)]
    L.or_pc_create_ras_sets.restype = P
    L.or_pc_create_learned.restype = P
    L.or_pc_apply.argtypes = [P, P, P]
    L.or_pc_destroy.argtypes = [P]
    L.or_pc_learned_stats.argtypes = [P, C.POINTER(C.c_long), C.POINTER(C.c_long)]
    L.or_cpr_weights.argtypes = [I, P, P, P, P]
    L.or_cpr_weights.restype = I
    L.or_cpr_extract_pressure.argtypes = [I, P, P, P, P, P]
    L.or_gmres.argtypes = [I, I, P, P, P, P, P, P, P, P, P]
    L.or_gmres.restype = I
    L.or_bicgstab.argtypes = [I, I, P, P, P, P, P, P, P, P, P]
    L.or_bicgstab.restype = I
    L.or_conv_nparams.restype = I
    L.or_conv_forward.argtypes = [I, I, I, P, P, P, I]
    L.or_conv_loss_grad.argtypes = [I, I, I, P, P, P, P, P, I]
    L.or_conv_loss_grad.restype = D
    L.or_adam_step.argtypes = [I, P, P, P, P, I, D, D, D, D]
    L.or_amg_defaults.argtypes = [P]
    L.or_amg_create.argtypes = [I, P, P, P, P, C.POINTER(I)]
    L.or_amg_create.restype = P
    L.or_amg_vcycle.argtypes = [P, P, P]
    L.or_amg_destroy.argtypes = [P]
    L.or_amg_strength.argtypes = [I, P, P, P, D, D, P, P]
    L.or_amg_strength.restype = I
    L.or_amg_nlevels.argtypes = [P]
    L.or_amg_nlevels.restype = I
    L.or_amg_level_size.argtypes = [P, I, C.POINTER(I), C.POINTER(I), C.POINTER(I),
                                    C.POINTER(I)]
    L.or_amg_level_get.argtypes = [P, I, P, P, P, P, P, P, P]
    L.or_pc_create_amg.argtypes = [I, I, I, P, P, P, P, C.POINTER(I)]
    L.or_pc_create_amg.restype = P
    L.or_pc_create_cpr.argtypes = [I, I, P, P, P, P, I, P, C.POINTER(I)]
    L.or_pc_create_cpr.restype = P
    L.or_gelu.argtypes = [D]
    L.or_gelu.restype = D
    L.or_bf16_round.argtypes = [C.c_float]
    L.or_bf16_round.restype = C.c_float
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        _lib = load(_SO)
    return _lib


def compile_variant(src_text: str, out_path: str) -> str:
    """Compile a modified copy of oracle.c (used by the tests that plant a
    mistake in the oracle and check that a pin catches it)."""
    d = os.path.dirname(out_path)
    cpath = os.path.join(d, "oracle_variant.c")
    with open(cpath, "w") as f:
        f.write(src_text)
    subprocess.check_call(
        ["gcc", "-O1", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
         "-I", _HERE, "-o", out_path, cpath, "-lm"])
    return out_path


def source() -> str:
    with open(_SRC) as f:
        return f.read()


class KrylovOpts(C.Structure):
    _fields_ = [("restart", C.c_int), ("maxit", C.c_int), ("rtol", C.c_double),
                ("atol", C.c_double), ("flexible", C.c_int), ("left", C.c_int),
                ("check_at_cycle_end", C.c_int), ("fixed_iters", C.c_int)]


class KrylovResult(C.Structure):
    _fields_ = [("iters", C.c_int), ("true_relres", C.c_double),
                ("restarts", C.c_int)]


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Matrix:
    """Block-CSR view of a generated system (bs = 1 for CSR)."""

    def __init__(self, rowptr, col, val, bs=1):
        self.rowptr = _i32(rowptr)
        self.col = _i32(col)
        self.bs = int(bs)
        self.val = _f64(val).reshape(-1)
        self.nb = self.rowptr.size - 1
        self.n = self.nb * self.bs

    @classmethod
    def from_system(cls, s):
        return cls(s["rowptr"], s["col"], s["val"], s.get("bs", 1))

    def args(self):
        return (self.nb, self.bs, _p(self.rowptr), _p(self.col), _p(self.val))


def spmv(A: Matrix, x):
    x = _f64(x)
    y = np.empty(A.n)
    lib().or_bsr_spmv(*A.args(), _p(x), _p(y))
    return y


def amxpby(A: Matrix, alpha, x, beta, y):
    x = _f64(x)
    y = _f64(y).copy()
    lib().or_bsr_amxpby(A.nb, A.bs, _p(A.rowptr), _p(A.col), _p(A.val),
                        alpha, _p(x), beta, _p(y))
    return y


def bilu0(A: Matrix):
    lu = np.empty_like(A.val)
    rc = lib().or_bilu0(*A.args(), _p(lu))
    return rc, lu


def bilu0_solve(A: Matrix, lu, b, part="both"):
    b = _f64(b)
    x = np.empty(A.n)
    lu = _f64(lu)
    f = {"both": lib().or_bilu0_solve, "lower": lib().or_bilu0_solve_lower,
         "upper": lib().or_bilu0_solve_upper}[part]
    f(A.nb, A.bs, _p(A.rowptr), _p(A.col), _p(lu), _p(b), _p(x))
    return x


def cpr_weights(A: Matrix):
    w = np.empty(3 * A.nb)
    rc = lib().or_cpr_weights(A.nb, _p(A.rowptr), _p(A.col), _p(A.val), _p(w))
    return rc, w


def cpr_pressure_matrix(A: Matrix, w):
    app = np.empty(A.rowptr[-1])
    w = _f64(w)
    lib().or_cpr_extract_pressure(A.nb, _p(A.rowptr), _p(A.col), _p(A.val),
                                  _p(w), _p(app))
    return app


class AmgOpts(C.Structure):
    _fields_ = [("strength", C.c_double), ("max_row_sum", C.c_double), ("trunc", C.c_double),
                ("max_levels", C.c_int), ("num_sweeps", C.c_int), ("gs_chunk", C.c_int),
                ("coarse_size", C.c_int)]

    @classmethod
    def make(cls, **kw):
        """Figure 34's defaults, with keyword overrides."""
        o = cls()
        lib().or_amg_defaults(C.byref(o))
        for k, v in kw.items():
            if k not in dict(cls._fields_):
                raise KeyError(k)
            setattr(o, k, v)
        return o


def amg_strength(A: Matrix, theta=0.5, max_row_sum=0.9):
    """Strong dependencies of every row as a CSR pattern (srp, sci)."""
    srp = np.empty(A.nb + 1, dtype=np.int32)
    sci = np.empty(max(1, int(A.rowptr[-1])), dtype=np.int32)
    m = lib().or_amg_strength(A.nb, _p(A.rowptr), _p(A.col), _p(A.val), float(theta),
                              float(max_row_sum), _p(srp), _p(sci))
    return srp, sci[:m].copy()


class AMG:
    """Oracle AMG hierarchy of a scalar matrix (Algorithm 3 on every level);
    vcycle(b) is Algorithm 4 from x = 0."""

    def __init__(self, A: Matrix, **opts):
        if A.bs != 1:
            raise ValueError("AMG takes a scalar matrix")
        self.A = A
        self.opts = AmgOpts.make(**opts)
        err = C.c_int(0)
        self.h = lib().or_amg_create(A.nb, _p(A.rowptr), _p(A.col), _p(A.val),
                                     C.byref(self.opts), C.byref(err))
        self.err = err.value
        if not self.h:
            raise RuntimeError(f"oracle AMG setup failed: {self.err}")

    def vcycle(self, b):
        b = _f64(b)
        x = np.empty(self.A.n)
        lib().or_amg_vcycle(self.h, _p(b), _p(x))
        return x

    @property
    def nlevels(self):
        return lib().or_amg_nlevels(self.h)

    def level(self, l):
        """dict(A=(rp, ci, a), cf, P=(rp, ci, v), n, nc); cf and P are None
        on the coarsest level"""
        n, nnz, nc, pnnz = (C.c_int() for _ in range(4))
        lib().or_amg_level_size(self.h, l, C.byref(n), C.byref(nnz), C.byref(nc),
                                C.byref(pnnz))
        n, nnz, nc, pnnz = n.value, nnz.value, nc.value, pnnz.value
        rp = np.empty(n + 1, dtype=np.int32)
        ci = np.empty(max(nnz, 1), dtype=np.int32)
        a = np.empty(max(nnz, 1))
        cf = np.empty(max(n, 1), dtype=np.int32)
        prp = np.empty(n + 1, dtype=np.int32)
        pci = np.empty(max(pnnz, 1), dtype=np.int32)
        pv = np.empty(max(pnnz, 1))
        lib().or_amg_level_get(self.h, l, _p(rp), _p(ci), _p(a), _p(cf), _p(prp), _p(pci),
                               _p(pv))
        coarse = l == self.nlevels - 1
        return dict(n=n, nc=nc, A=(rp, ci[:nnz], a[:nnz]),
                    cf=None if coarse else cf[:n],
                    P=None if coarse else (prp, pci[:pnnz], pv[:pnnz]))

    def __del__(self):
        if getattr(self, "h", None):
            lib().or_amg_destroy(self.h)
            self.h = None


class PC:
    """Oracle preconditioner: kind in none/bilu0/cpr_pf/cpr_fp/cpr_fpf/
    cpr_ffpf, precision
    f64/f32/bf16, p_sweeps = ILU(0) sweeps of the CPR pressure stage."""

    def __init__(self, A: Matrix, kind="bilu0", prec="f64", p_sweeps=4):
        self.A = A
        err = C.c_int(0)
        self.h = lib().or_pc_create(PC_KIND[kind], *A.args(), PREC[prec],
                                    int(p_sweeps), C.byref(err))
        self.err = err.value
        if not self.h:
            raise RuntimeError(f"oracle PC setup failed: {self.err}")

    @classmethod
    def learned(cls, base: "PC", grid, params, lnk, bf16=True):
        obj = cls.__new__(cls)
        obj.A = base.A
        obj.err = 0
        params = _f64(params)
        lnk = _f64(lnk)
        nx, ny, nz = grid
        obj.h = lib().or_pc_create_learned(base.h, nx, ny, nz, _p(params),
                                           _p(lnk), int(bf16))
        base.h = None      # ownership moved
        return obj

    @classmethod
    def amg(cls, A: "Matrix", kind="amg", **opts):
        """AMG preconditioners (FP64): kind "amg", one V-cycle on a scalar
        matrix; or a CPR kind whose pressure stage is one V-cycle on A_pp."""
        obj = cls.__new__(cls)
        obj.A = A
        obj._opts = AmgOpts.make(**opts)
        err = C.c_int(0)
        obj.h = lib().or_pc_create_amg(PC_KIND[kind], *A.args(), C.byref(obj._opts),
                                       C.byref(err))
        obj.err = err.value
        if not obj.h:
            raise RuntimeError(f"oracle AMG setup failed: {obj.err}")
        return obj

    @classmethod
    def cpr(cls, A: "Matrix", kind="cpr_fpf", amg=None, p_sweeps=4, full=None):
        """FP64 CPR whose pressure stage is one AMG V-cycle (amg = dict of
        AMG options, {} for the defaults) or p_sweeps ILU(0) sweeps, and
        whose full-system stage R(A)^-1 is the preconditioner `full` (a PC,
        e.g. RAS; it is taken over) or block ILU(0)."""
        obj = cls.__new__(cls)
        obj.A = A
        obj._opts = None if amg is None else AmgOpts.make(**amg)
        fh = None
        if full is not None:
            fh, full.h = full.h, None      # ownership moves to the CPR object
        err = C.c_int(0)
        obj.h = lib().or_pc_create_cpr(PC_KIND[kind], A.nb, _p(A.rowptr), _p(A.col), _p(A.val),
                                       None if obj._opts is None else C.byref(obj._opts),
                                       int(p_sweeps), fh, C.byref(err))
        obj.err = err.value
        if not obj.h:
            raise RuntimeError(f"oracle CPR setup failed: {obj.err}")
        return obj

    @classmethod
    def ras(cls, A: "Matrix", starts, overlap=1):
        """Restricted additive Schwarz with block ILU(0) subdomain solves;
        `starts` = block-row offsets of the owned ranges (0 .. nb)."""
        obj = cls.__new__(cls)
        obj.A = A
        st = _i32(starts)
        obj._starts = st
        err = C.c_int(0)
        obj.h = lib().or_pc_create_ras(*A.args(), int(st.size - 1), _p(st), int(overlap),
                                       C.byref(err))
        obj.err = err.value
        if not obj.h:
            raise RuntimeError(f"oracle RAS setup failed: {obj.err}")
        return obj

    @classmethod
    def ras_part(cls, A: "Matrix", part, overlap=1):
        """RAS with block row r owned by subdomain part[r]."""
        obj = cls.__new__(cls)
        obj.A = A
        pa = _i32(part)
        obj._part = pa
        err = C.c_int(0)
        obj.h = lib().or_pc_create_ras_part(*A.args(), int(pa.max()) + 1, _p(pa), int(overlap),
                                            C.byref(err))
        obj.err = err.value
        if not obj.h:
            raise RuntimeError(f"oracle RAS setup failed: {obj.err}")
        return obj

    @classmethod
    def ras_sets(cls, A: "Matrix", part, sets):
        """RAS with block row r owned by part[r] and subdomain s solving on
        the block rows sets[s] (ascending, holding its owned rows)."""
        obj = cls.__new__(cls)
        obj.A = A
        pa = _i32(part)
        ptr = _i32(np.concatenate([[0], np.cumsum([len(x) for x in sets])]))
        flat = _i32(np.concatenate([np.asarray(x) for x in sets]))
        obj._keep = (pa, ptr, flat)
        err = C.c_int(0)
        obj.h = lib().or_pc_create_ras_sets(*A.args(), len(sets), _p(pa), _p(ptr), _p(flat),
                                            C.byref(err))
        obj.err = err.value
        if not obj.h:
            raise RuntimeError(f"oracle RAS setup failed: {obj.err}")
        return obj

    def apply(self, v):
        v = _f64(v)
        z = np.empty(self.A.n)
        lib().or_pc_apply(self.h, _p(v), _p(z))
        return z

    def learned_stats(self):
        a, f = C.c_long(0), C.c_long(0)
        lib().or_pc_learned_stats(self.h, C.byref(a), C.byref(f))
        return a.value, f.value

    def __del__(self):
        if getattr(self, "h", None):
            lib().or_pc_destroy(self.h)
            self.h = None


def _solve(fn, A, pc, b, x0, restart, maxit, rtol, atol, flexible, left,
           check_at_cycle_end, fixed_iters, hist):
    b = _f64(b)
    x = np.zeros(A.n) if x0 is None else _f64(x0).copy()
    o = KrylovOpts(int(restart), int(maxit), float(rtol), float(atol),
                   int(flexible), int(left), int(check_at_cycle_end),
                   int(fixed_iters))
    r = KrylovResult()
    h = np.zeros(int(maxit) + 2) if hist else None
    rc = fn(*A.args(), C.c_void_p(pc.h), _p(b), _p(x), C.byref(o), C.byref(r),
            _p(h) if hist else None)
    out = dict(status=rc, x=x, iters=r.iters, relres=r.true_relres,
               restarts=r.restarts)
    if hist:
        out["hist"] = h[:r.iters + 1]
    return out


def gmres(A, pc, b, x0=None, restart=30, maxit=500, rtol=1e-6, atol=0.0,
          flexible=False, left=False, check_at_cycle_end=False,
          fixed_iters=False, hist=False):
    return _solve(lib().or_gmres, A, pc, b, x0, restart, maxit, rtol, atol,
                  flexible, left, check_at_cycle_end, fixed_iters, hist)


def lgmres(A, pc, b, x0=None, restart=30, aug_k=2, maxit=500, rtol=1e-6, atol=0.0,
           fixed_iters=False, hist=False):
    """LGMRES(restart, aug_k), right preconditioned, flexible storage."""
    fn = lambda *args: lib().or_lgmres(*args[:-2], int(aug_k), *args[-2:])
    return _solve(fn, A, pc, b, x0, restart, maxit, rtol, atol, True, False, False,
                  fixed_iters, hist)


def pcg(A, pc, b, x0=None, maxit=500, rtol=1e-6, atol=0.0, fixed_iters=False, hist=False):
    """Preconditioned CG (Algorithm 2) for SPD A and M."""
    return _solve(lib().or_pcg, A, pc, b, x0, 0, maxit, rtol, atol, False, False, False,
                  fixed_iters, hist)


def bicgstab(A, pc, b, x0=None, maxit=500, rtol=1e-6, atol=0.0,
             fixed_iters=False, hist=False):
    return _solve(lib().or_bicgstab, A, pc, b, x0, 0, maxit, rtol, atol,
                  False, False, False, fixed_iters, hist)


# ---- learned-stage network -------------------------------------------------
CONV_CH = (4, 32, 32, 32, 3)


def conv_nparams():
    return lib().or_conv_nparams()


def conv_forward(grid, params, inp, bf16=False):
    nx, ny, nz = grid
    params = _f64(params)
    inp = _f64(inp)
    out = np.empty(3 * nx * ny * nz)
    lib().or_conv_forward(nx, ny, nz, _p(params), _p(inp), _p(out), int(bf16))
    return out


def conv_loss_grad(grid, params, inp, target, bf16=False, want_dinput=False):
    nx, ny, nz = grid
    params = _f64(params)
    inp = _f64(inp)
    target = _f64(target)
    grad = np.empty(params.size)
    din = np.empty(inp.size) if want_dinput else None
    loss = lib().or_conv_loss_grad(nx, ny, nz, _p(params), _p(inp), _p(target),
                                   _p(grad), _p(din) if want_dinput else None,
                                   int(bf16))
    return (loss, grad, din) if want_dinput else (loss, grad)


def adam_step(params, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999,
              eps=1e-8):
    params = _f64(params).copy()
    m = _f64(m).copy()
    v = _f64(v).copy()
    grad = _f64(grad)
    lib().or_adam_step(params.size, _p(params), _p(grad), _p(m), _p(v), int(t),
                       lr, beta1, beta2, eps)
    return params, m, v


def gelu(x):
    return lib().or_gelu(float(x))


def bf16_round(x):
    return float(lib().or_bf16_round(float(x)))
