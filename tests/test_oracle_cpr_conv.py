"""Pins of the oracle's CPR multi-stage preconditioners with quasi-IMPES
decoupling (eqs. (5)-(9), Algorithms 5-8), their reduced-precision
emulation, and the learned stage (conv net, Adam, apply with fallback)."""
import os

import numpy as np
import pytest

import oracle
import reservoir_inputs as ri
from tests._helpers import bsr_from_dense, dense, dense_from_bsr, lu_dense_from_factor, relerr

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---- C8 quasi-IMPES and CPR --------------------------------------------------
def test_quasi_impes_weights_zero_secondary_columns():
    s = ri.blackoil_system(5, 4, 3, seed=1)
    A = oracle.Matrix.from_system(s)
    rc, w = oracle.cpr_weights(A)
    assert rc == 0
    blocks = A.val.reshape(-1, 3, 3)
    for i in range(A.nb):
        p = [q for q in range(A.rowptr[i], A.rowptr[i + 1]) if A.col[q] == i][0]
        row = w[3 * i:3 * i + 3] @ blocks[p]
        assert w[3 * i] == 1.0
        assert np.all(np.abs(row[1:]) <= 1e-15 * np.abs(blocks[p]).max() * 4)


def test_pressure_matrix_is_decoupled_operator_on_pressure_vectors():
    # (A_pp p)_i must equal w_i^T (A Pi_p p)_i for every p
    s = ri.blackoil_system(4, 3, 3, seed=2)
    A = oracle.Matrix.from_system(s)
    rc, w = oracle.cpr_weights(A)
    app = oracle.cpr_pressure_matrix(A, w)
    P = oracle.Matrix(A.rowptr, A.col, app, 1)
    D = dense(s)
    rng = np.random.default_rng(0)
    for _ in range(3):
        p = rng.standard_normal(A.nb)
        x = np.zeros(A.n)
        x[0::3] = p
        Ax = (D @ x).reshape(-1, 3)
        ref = np.einsum("ij,ij->i", w.reshape(-1, 3), Ax)
        assert relerr(oracle.spmv(P, p), ref) < 1e-14


def _decoupled_1d(nb=15, seed=0):
    """Block tridiagonal system whose secondary unknowns only see their own
    diagonal: A_ij = diag(a_ij, 0, 0) off the diagonal."""
    rng = np.random.default_rng(seed)
    n = 3 * nb
    D = np.zeros((n, n))
    for i in range(nb):
        D[3*i, 3*i] = 4.0 + rng.random()
        D[3*i+1, 3*i+1] = 2.0 + rng.random()
        D[3*i+2, 3*i+2] = 2.0 + rng.random()
        D[3*i, 3*i+1] = 0.3 * rng.random()      # pressure row couples
        D[3*i, 3*i+2] = 0.3 * rng.random()
        for j in (i - 1, i + 1):
            if 0 <= j < nb:
                D[3*i, 3*j] = -1.0 - rng.random()
    return D


CPR_KINDS = ["cpr_pf", "cpr_fp", "cpr_fpf", "cpr_ffpf"]


@pytest.mark.parametrize("kind", CPR_KINDS)
def test_cpr_exact_when_stages_are_exact(kind):
    D = _decoupled_1d()
    s = bsr_from_dense(D, 3)
    A = oracle.Matrix.from_system(s)
    pc = oracle.PC(A, kind, p_sweeps=1)
    v = np.random.default_rng(1).standard_normal(A.n)
    assert relerr(pc.apply(v), np.linalg.solve(D, v)) < 1e-12
    r = oracle.gmres(A, pc, v, restart=30, maxit=10, rtol=1e-10, flexible=True)
    assert r["iters"] == 1


def test_pressure_sweeps_after_exact_first_sweep_change_nothing():
    # tridiagonal A_pp (1D grid): sweep 1 is exact, sweeps 2-4 add zero
    s = ri.blackoil_system(25, 1, 1, seed=3)
    A = oracle.Matrix.from_system(s)
    v = np.random.default_rng(2).standard_normal(A.n)
    z1 = oracle.PC(A, "cpr_pf", p_sweeps=1).apply(v)
    z4 = oracle.PC(A, "cpr_pf", p_sweeps=4).apply(v)
    assert relerr(z4, z1) < 1e-13


def test_converged_pressure_stage_solves_pressure_only_systems():
    # v = A Pi_p p*: the decoupled pressure residual is A_pp p*, so a
    # converged pressure stage returns p* and the second stage sees r = 0
    s = ri.blackoil_system(6, 6, 6, seed=4)
    A = oracle.Matrix.from_system(s)
    rng = np.random.default_rng(5)
    pstar = rng.standard_normal(A.nb)
    x = np.zeros(A.n)
    x[0::3] = pstar
    v = dense(s) @ x
    z = oracle.PC(A, "cpr_pf", p_sweeps=200).apply(v)
    assert relerr(z, x) < 1e-10
    z1 = oracle.PC(A, "cpr_pf", p_sweeps=1).apply(v)
    assert relerr(z1, x) > 1e-6


# stage order of each variant, first applied first (Algorithms 5-8; the
# PF variant in the two-stage reading)
STAGES = {"cpr_pf": "PF", "cpr_fp": "FP", "cpr_fpf": "FPF", "cpr_ffpf": "FFPF"}


@pytest.mark.parametrize("p_sweeps", [1, 3])
@pytest.mark.parametrize("kind", CPR_KINDS)
def test_cpr_error_propagator_is_product_of_stage_propagators(kind, p_sweeps):
    """Each stage x <- x + B (f - A x) multiplies the error by (I - B A), so
    the preconditioner is M^-1 = (I - prod_k (I - B_k A)) A^-1, with the
    last stage leftmost.  B_F = (L U)^-1 from the dense block factor;
    B_P = Pi_p S Pi_r W with S the closed form of s stationary sweeps from
    zero, S = (I - (I - M_p^-1 A_pp)^s) A_pp^-1."""
    s = ri.blackoil_system(3, 3, 2, seed=11)
    A = oracle.Matrix.from_system(s)
    D = dense(s)
    n, nb = A.n, A.nb
    rc, lu = oracle.bilu0(A)
    assert rc == 0
    L, U = lu_dense_from_factor(A.rowptr, A.col, lu, 3)
    BF = np.linalg.inv(L @ U)
    rc, w = oracle.cpr_weights(A)
    app = oracle.cpr_pressure_matrix(A, w)
    P = oracle.Matrix(A.rowptr, A.col, app, 1)
    rc, plu = oracle.bilu0(P)
    assert rc == 0
    Lp, Up = lu_dense_from_factor(A.rowptr, A.col, plu, 1)
    App = dense_from_bsr(A.rowptr, A.col, app, 1)
    G = np.eye(nb) - np.linalg.solve(Lp @ Up, App)
    S = (np.eye(nb) - np.linalg.matrix_power(G, p_sweeps)) @ np.linalg.inv(App)
    R = np.zeros((nb, n))
    Pi = np.zeros((n, nb))
    for i in range(nb):
        R[i, 3 * i:3 * i + 3] = w[3 * i:3 * i + 3]
        Pi[3 * i, i] = 1.0
    BP = Pi @ S @ R
    E = np.eye(n)
    for st in STAGES[kind]:
        E = (np.eye(n) - (BF if st == "F" else BP) @ D) @ E
    Minv = (np.eye(n) - E) @ np.linalg.inv(D)
    v = np.random.default_rng(12).standard_normal(n)
    z = oracle.PC(A, kind, p_sweeps=p_sweeps).apply(v)
    assert relerr(z, Minv @ v) < 1e-11


def test_cpr_variants_differ():
    # the four step sequences are different operators on a generic system
    s = ri.blackoil_system(5, 4, 3, seed=13)
    A = oracle.Matrix.from_system(s)
    v = np.random.default_rng(14).standard_normal(A.n)
    zs = [oracle.PC(A, k).apply(v) for k in CPR_KINDS]
    for a in range(4):
        for b in range(a + 1, 4):
            assert relerr(zs[a], zs[b]) > 1e-6


@pytest.mark.parametrize("kind", ["bilu0"] + CPR_KINDS)
def test_reduced_precision_apply_close_to_fp64(kind):
    s = ri.blackoil_system(8, 8, 8, seed=6)
    A = oracle.Matrix.from_system(s)
    v = np.random.default_rng(3).standard_normal(A.n)
    z64 = oracle.PC(A, kind, "f64").apply(v)
    z32 = oracle.PC(A, kind, "f32").apply(v)
    zb = oracle.PC(A, kind, "bf16").apply(v)
    assert 0 < relerr(z32, z64) < 1e-4
    assert relerr(z32, z64) < relerr(zb, z64) < 5e-2


def test_mixed_precision_fgmres_reaches_fp64_true_residual():
    s = ri.blackoil_system(10, 10, 10, seed=7)
    A = oracle.Matrix.from_system(s)
    for prec in ("f32", "bf16"):
        r = oracle.gmres(A, oracle.PC(A, "bilu0", prec), s["b"], restart=30,
                         maxit=2000, rtol=1e-8, flexible=True)
        assert r["status"] == 0 and r["relres"] <= 1e-8


# ---- C10 conv net ------------------------------------------------------------
def _params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    ch = oracle.CONV_CH
    out = []
    for l in range(4):
        fan = ch[l] * 27
        bound = 1.0 / np.sqrt(fan)
        out.append(scale * rng.uniform(-bound, bound, ch[l + 1] * fan))
        out.append(scale * rng.uniform(-bound, bound, ch[l + 1]))
    return np.concatenate(out)


def test_nparams():
    assert oracle.conv_nparams() == 4*32*27+32 + 2*(32*32*27+32) + 32*3*27+3


def test_gelu_closed_forms():
    with open(os.path.join(GOLDEN, "gelu_phi.txt")) as f:
        for ln in f:
            if ln.strip() and not ln.startswith("#"):
                x, y = map(float, ln.split())
                assert abs(oracle.gelu(x) - y) <= 1e-15 * max(1.0, abs(y))


def test_conv_finite_differences():
    grid = (3, 3, 2)
    cells = 18
    rng = np.random.default_rng(0)
    prm = _params(1, scale=2.0)
    inp = rng.standard_normal(4 * cells)
    tgt = rng.standard_normal(3 * cells)
    loss, grad, din = oracle.conv_loss_grad(grid, prm, inp, tgt, want_dinput=True)
    eps = 1e-6
    idx = list(rng.choice(prm.size, 40, replace=False)) + list(range(prm.size - 3, prm.size))
    for i in idx:
        pp = prm.copy(); pp[i] += eps
        pm = prm.copy(); pm[i] -= eps
        fd = (oracle.conv_loss_grad(grid, pp, inp, tgt)[0] - oracle.conv_loss_grad(grid, pm, inp, tgt)[0]) / (2 * eps)
        assert abs(fd - grad[i]) <= 1e-6 * max(abs(grad[i]), 1e-3)
    for i in rng.choice(inp.size, 10, replace=False):
        ip = inp.copy(); ip[i] += eps
        im = inp.copy(); im[i] -= eps
        fd = (oracle.conv_loss_grad(grid, prm, ip, tgt)[0] - oracle.conv_loss_grad(grid, prm, im, tgt)[0]) / (2 * eps)
        assert abs(fd - din[i]) <= 1e-6 * max(abs(din[i]), 1e-3)


def _identity_params():
    ch = oracle.CONV_CH
    out = []
    for l in range(4):
        W = np.zeros((ch[l + 1], ch[l], 27))
        for c in range(min(ch[l], ch[l + 1])):
            W[c, c, 13] = 1.0         # centre tap
        out.append(W.ravel())
        out.append(np.zeros(ch[l + 1]))
    return np.concatenate(out)


def test_conv_delta_kernels_give_identity_for_large_inputs():
    # GELU(x) = x Phi(x) equals x to double precision for x >= 10
    grid = (4, 3, 3)
    cells = 36
    inp = 10.0 + np.random.default_rng(1).random(4 * cells)
    out = oracle.conv_forward(grid, _identity_params(), inp)
    assert relerr(out, inp[:3 * cells]) < 1e-15


def test_conv_translation_equivariance():
    grid = (14, 11, 11)
    nx, ny, nz = grid
    cells = nx * ny * nz
    prm = _params(2)
    rng = np.random.default_rng(2)
    base = np.zeros((4, nz, ny, nx))
    base[:, 4:7, 4:7, 4:8] = rng.standard_normal((4, 3, 3, 4))
    shifted = np.roll(base, 1, axis=3)
    o1 = oracle.conv_forward(grid, prm, base.ravel()).reshape(3, nz, ny, nx)
    o2 = oracle.conv_forward(grid, prm, shifted.ravel()).reshape(3, nz, ny, nx)
    # receptive field radius 4: cells at least 4 from every face
    assert np.allclose(o2[:, 4:-4, 4:-4, 5:-4], o1[:, 4:-4, 4:-4, 4:-5], rtol=0, atol=1e-14)


def test_conv_bf16_emulation_close():
    grid = (5, 4, 3)
    cells = 60
    prm = _params(3)
    inp = np.random.default_rng(3).standard_normal(4 * cells)
    a = oracle.conv_forward(grid, prm, inp)
    b = oracle.conv_forward(grid, prm, inp, bf16=True)
    assert 0 < relerr(b, a) < 2e-2


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(4)
    p0 = rng.standard_normal(50)
    g = rng.standard_normal(50)
    p1, m, v = oracle.adam_step(p0, g, np.zeros(50), np.zeros(50), 1, lr=1e-3)
    # bias-corrected moments of the first step are g and g^2
    assert np.allclose(p1, p0 - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


# ---- C11 learned stage with fallback ----------------------------------------------
def test_learned_stage_zero_net_falls_back_bit_exactly():
    s = ri.blackoil_system(6, 5, 4, seed=9)
    A = oracle.Matrix.from_system(s)
    v = np.random.default_rng(5).standard_normal(A.n)
    base = oracle.PC(A, "bilu0")
    z_base = base.apply(v)
    zero = np.zeros(oracle.conv_nparams())
    pc = oracle.PC.learned(oracle.PC(A, "bilu0"), s["grid"], zero, s["lnk"])
    z = pc.apply(v)
    assert np.array_equal(z, z_base)
    assert pc.learned_stats() == (1, 1)
    nan = np.full(oracle.conv_nparams(), np.nan)
    pc2 = oracle.PC.learned(oracle.PC(A, "bilu0"), s["grid"], nan, s["lnk"])
    assert np.array_equal(pc2.apply(v), z_base)
    assert pc2.learned_stats() == (1, 1)


def test_learned_stage_zero_net_solve_equals_plain_fgmres():
    s = ri.blackoil_system(6, 6, 6, seed=10)
    A = oracle.Matrix.from_system(s)
    zero = np.zeros(oracle.conv_nparams())
    pc = oracle.PC.learned(oracle.PC(A, "bilu0"), s["grid"], zero, s["lnk"])
    a = oracle.gmres(A, pc, s["b"], restart=30, maxit=500, rtol=1e-8, flexible=True)
    b = oracle.gmres(A, oracle.PC(A, "bilu0"), s["b"], restart=30, maxit=500, rtol=1e-8, flexible=True)
    assert a["iters"] == b["iters"] and np.array_equal(a["x"], b["x"])


def test_learned_stage_accepts_a_useful_correction():
    # a "network" that outputs the exact error of z1 (built by hand here
    # as the identity on r1/s, valid when A^-1 r1 ~ r1 is not needed:
    # instead check acceptance logic with the exact correction injected
    # through a diagonal system where BILU(0) is exact up to scaling)
    D = np.diag(np.linspace(1.0, 2.0, 3 * 8))
    s = bsr_from_dense(D, 3)
    A = oracle.Matrix.from_system(s)
    # BILU(0) on a diagonal matrix is exact, so r1 = 0 and the stage must
    # leave z1 untouched (s = 0 path)
    pc = oracle.PC.learned(oracle.PC(A, "bilu0"), (2, 2, 2), _params(5), np.zeros(8))
    v = np.arange(24.0)
    assert relerr(pc.apply(v), v / np.diag(D)) < 1e-15
    assert pc.learned_stats()[1] == 1
