"""The C-ABI library loads without a GPU and exports every function that
include/krylov.h declares; the Python binding declares the same set."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "krylov.h")
LIB = os.path.join(ROOT, "paper_1701_05913_amd", "libkrylov.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set()
    for m in re.finditer(r"^\s*(?!typedef)[A-Za-z_][\w\s\*]*?\b([A-Z]\w+)\s*\(", src, flags=re.M):
        names.add(m.group(1))
    return names


def test_header_parses():
    names = declared_functions()
    for must in ["MapCreate", "VecAXPBY", "MatCreateBSR", "MatVecAMXPBY", "SolverSolve",
                 "SolverSetPC", "LastError", "KernelTimingQuery"]:
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_function():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in sorted(declared_functions()) if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_matches_header():
    import paper_1701_05913_amd as K
    assert set(K.exported_symbols()) == declared_functions()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_host_side_argument_errors_without_gpu():
    # calls that fail before touching the GPU
    import paper_1701_05913_amd as K
    with pytest.raises(K.KrylovError):
        K.MapCreate(5, 5)                       # eq. (2): ilower < iupper
    m = K.MapCreateLocal(10)
    assert K.MapGetNlocal(m) == 10
    with pytest.raises(K.KrylovError):
        K.SolverCreate(7, K.KRY_PC_NONE, m)      # unknown solver type
    s = K.SolverCreate(K.KRY_GMRES, K.KRY_PC_ILU0, m)
    with pytest.raises(K.KrylovError):
        K.SolverSetRestart(s, 0)
    with pytest.raises(K.KrylovError):
        K.SolverSetAugk(s, -1)                   # aug_k < 0
    with pytest.raises(K.KrylovError):
        K.SolverSetAugk(s, 40)                   # restart 30 + aug_k > 63
    K.SolverSetAugk(s, 2)                        # LGMRES(30, 2)
    with pytest.raises(K.KrylovError):
        K.SolverAssemble(s)                      # no matrix
    # the RAS, AMG and CPR-stage setters check their arguments on the host
    for bad in ((0, 1, 1, 1), (1, 0, 1, 1), (1, 1, 0, 1), (1, 1, 1, -1)):
        with pytest.raises(K.KrylovError):
            K.SolverSetRASBoxes(s, *bad)
    for bad in ((0, 1), (2, -1)):
        with pytest.raises(K.KrylovError):
            K.SolverSetRAS(s, *bad)
    for bad in ((0, 2, 4), (8, 0, 4)):
        with pytest.raises(K.KrylovError):
            K.SolverSetAMG(s, *bad)
    with pytest.raises(K.KrylovError):
        K.SolverSetCPRPressure(s, 2)
    with pytest.raises(K.KrylovError):
        K.SolverSetCPRFull(s, 2)
    with pytest.raises(K.KrylovError):
        K.SolverSetOrthog(s, 2)                  # neither AUTO nor CGS2
    K.SolverSetOrthog(s, K.KRY_ORTHO_CGS2)
    K.SolverSetRASBoxes(s, 2, 2, 2, 1)
    K.SolverSetAMG(s, 6, 1, 8)
    K.SolverSetCPRPressure(s, K.KRY_CPR_P_AMG)
    K.SolverSetCPRFull(s, K.KRY_CPR_F_RAS)
    with pytest.raises(K.KrylovError):
        K.SolverGetAMGLevels(s)                  # nothing assembled
    # the timing selection is host state only
    K.KernelTimingSelect("ilu_bwd_bsr3_f64,spmv_bsr3")
    K.KernelTimingSelect(["cgs2"])
    K.KernelTimingSelect(None)
    K.KernelTimingSample(4)
    K.KernelTimingSample(1)
    with pytest.raises(K.KrylovError):
        K.KernelTimingSample(0)
    K.SolverDestroy(s)
    K.MapDestroy(m)
