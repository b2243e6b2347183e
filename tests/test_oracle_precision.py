"""Closed-form pins of the oracle's reduced-precision emulation (mixed
precision extension; the sweeps of eq. (3) in float, factors stored in
float or bfloat16, diagonal-block inverses kept in float, the CPR pressure
stage of Algorithms 5-6 in float, and the bfloat16 operands of the
learned stage's conv layers).

Every expected value below is derived by hand from the rounding rules
(binary32: 24 significant bits, spacing 2^-23 on [1, 2) and 2^-24 on
[1/2, 1); bfloat16: 8 significant bits, spacing 2^-7 on [1, 2);
round to nearest, ties to even), on tiny systems chosen so that the FP64,
FP32 and BF16 answers are three different exact numbers.  A dropped
rounding step, a wider accumulator or a factor rounded to the wrong format
moves the result off these values.
"""
import numpy as np

import oracle

E11, E12, E24 = 2.0 ** -11, 2.0 ** -12, 2.0 ** -24


def _scalar(rows):
    """CSR matrix (bs = 1) from a dense list of rows, pattern = nonzeros
    plus the diagonal."""
    rp, ci, va = [0], [], []
    for i, row in enumerate(rows):
        for j, a in enumerate(row):
            if a != 0.0 or i == j:
                ci.append(j)
                va.append(a)
        rp.append(len(ci))
    return oracle.Matrix(rp, ci, va, bs=1)


def test_forward_sweep_accumulates_in_float():
    # L = [[1, 0], [l, 1]], l = 1 + 2^-12, b = (1 + 2^-12, 1 + 2^-11).
    # y2 = b2 - l y1 with l y1 = 1 + 2^-11 + 2^-24 exactly.
    #  FP64: y2 = -2^-24.
    #  FP32: fl(l y1) is a tie between 1 + 2^-11 and its odd neighbour and
    #        goes to 1 + 2^-11, so y2 = 0 exactly.  (A double accumulator
    #        rounded once at the end gives -2^-24.)
    #  BF16 factors: l rounds to 1 (2^-12 is below half of 2^-7), so
    #        y2 = (1 + 2^-11) - (1 + 2^-12) = 2^-12 exactly.
    l = 1.0 + E12
    A = _scalar([[1.0, 0.0], [l, 1.0]])
    b = np.array([1.0 + E12, 1.0 + E11])
    z64 = oracle.PC(A, "ilu0", "f64").apply(b)
    z32 = oracle.PC(A, "ilu0", "f32").apply(b)
    zbf = oracle.PC(A, "ilu0", "bf16").apply(b)
    assert z64.tolist() == [1.0 + E12, -E24]
    assert z32.tolist() == [1.0 + E12, 0.0]
    assert zbf.tolist() == [1.0 + E12, E12]


def test_backward_sweep_accumulates_in_float():
    # U = [[1, u], [0, 1]], u = 1 + 2^-12, b = (1 + 2^-11, 1 + 2^-12):
    # x2 = 1 + 2^-12, x1 = b1 - u x2, the mirror image of the forward pin.
    u = 1.0 + E12
    A = _scalar([[1.0, u], [0.0, 1.0]])
    b = np.array([1.0 + E11, 1.0 + E12])
    assert oracle.PC(A, "ilu0", "f64").apply(b).tolist() == [-E24, 1.0 + E12]
    assert oracle.PC(A, "ilu0", "f32").apply(b).tolist() == [0.0, 1.0 + E12]
    assert oracle.PC(A, "ilu0", "bf16").apply(b).tolist() == [E12, 1.0 + E12]


def test_diagonal_inverse_kept_in_float_for_bf16_factors():
    # A = [d], d = 1 + 2^-12: 1/d = 1 - 2^-12 + 2^-24 - 2^-36 + ...
    # FP32 keeps 1 - 2^-12 + 2^-24 (spacing 2^-24 below 1); bfloat16 would
    # round it to 1.  The BF16 variant stores only the off-diagonal factors
    # in bfloat16, so both reduced variants give 1 - 2^-12 + 2^-24.
    d = 1.0 + E12
    A = _scalar([[d]])
    b = np.array([1.0])
    assert oracle.PC(A, "ilu0", "f64").apply(b)[0] == 1.0 / d
    assert oracle.PC(A, "ilu0", "f32").apply(b)[0] == 1.0 - E12 + E24
    assert oracle.PC(A, "ilu0", "bf16").apply(b)[0] == 1.0 - E12 + E24


def test_bf16_rounds_off_diagonal_blocks_of_3x3_factors():
    # two cells, one 3x3 block below the diagonal: the same numbers as the
    # scalar forward pin in each of the three block rows (block = l I)
    l = 1.0 + E12
    I3 = np.eye(3)
    rp, ci = [0, 1, 3], [0, 0, 1]
    va = np.concatenate([I3.ravel(), (l * I3).ravel(), I3.ravel()])
    A = oracle.Matrix(rp, ci, va, bs=3)
    b = np.array([1.0 + E12] * 3 + [1.0 + E11] * 3)
    assert oracle.PC(A, "bilu0", "f64").apply(b)[3:].tolist() == [-E24] * 3
    assert oracle.PC(A, "bilu0", "f32").apply(b)[3:].tolist() == [0.0] * 3
    assert oracle.PC(A, "bilu0", "bf16").apply(b)[3:].tolist() == [E12] * 3


def _cpr_two_cells():
    # Two cells of a 1D grid, 3x3 blocks.  Diagonal blocks I (so the
    # quasi-IMPES weights are w = (1, 0, 0) and the pressure rows are
    # decoupled from the secondary unknowns); the one off-diagonal block
    # A_21 couples pressure to pressure only, with l = 1 + 2^-12.  The
    # pressure matrix is then A_pp = [[1, 0], [l, 1]], its ILU(0) is exact.
    l = 1.0 + E12
    B = np.zeros((3, 3))
    B[0, 0] = l
    rp, ci = [0, 1, 3], [0, 0, 1]
    va = np.concatenate([np.eye(3).ravel(), B.ravel(), np.eye(3).ravel()])
    return oracle.Matrix(rp, ci, va, bs=3)


def test_cpr_pf_pressure_stage_in_float():
    # v = pressure (1 + 2^-12, 1 + 2^-11), secondary 0.  CPR-PF:
    # p = 4 ILU(0) sweeps on A_pp from 0; z = Pi_p p + BILU^-1 (v - A Pi_p p).
    #  FP64: p = A_pp^-1 v_p = (1 + 2^-12, -2^-24), and the second stage
    #        sees a zero residual: z = (1 + 2^-12, 0, 0, -2^-24, 0, 0).
    #  FP32: sweep 1 gives p2 = 0 (the forward pin); the float residual of
    #        sweeps 2-4, r2 - (fl(l p1) + p2), is exactly 0, so p stays;
    #        the second stage's float residual is 0 too: z_p = (1 + 2^-12, 0).
    #        (A double accumulator in the stage's residual sees -2^-24 and
    #        moves p2 to -2^-24.)
    A = _cpr_two_cells()
    v = np.array([1.0 + E12, 0.0, 0.0, 1.0 + E11, 0.0, 0.0])
    z64 = oracle.PC(A, "cpr_pf", "f64").apply(v)
    z32 = oracle.PC(A, "cpr_pf", "f32").apply(v)
    assert z64.tolist() == [1.0 + E12, 0.0, 0.0, -E24, 0.0, 0.0]
    assert z32.tolist() == [1.0 + E12, 0.0, 0.0, 0.0, 0.0, 0.0]


def test_cpr_pf_pressure_sweeps_two_to_four_use_float_residual():
    # Same system, sweep count 2..4 must not change the FP32 answer, and a
    # single sweep already gives it (ILU(0) of A_pp is exact, so extra
    # sweeps only see the float residual, which is exactly zero here)
    A = _cpr_two_cells()
    v = np.array([1.0 + E12, 0.0, 0.0, 1.0 + E11, 0.0, 0.0])
    for sweeps in (1, 2, 4):
        z = oracle.PC(A, "cpr_pf", "f32", p_sweeps=sweeps).apply(v)
        assert z.tolist() == [1.0 + E12, 0.0, 0.0, 0.0, 0.0, 0.0]


def _delta_net(bias1, bias4):
    # 4 -> 32 -> 32 -> 32 -> 3 network whose channel 0 passes the input's
    # channel 0 through centre taps of weight 1; every other weight is 0
    ch = oracle.CONV_CH
    parts = []
    for l in range(4):
        W = np.zeros((ch[l + 1], ch[l], 27))
        W[0, 0, 13] = 1.0                     # centre tap (dz, dy, dx) = 0
        b = np.zeros(ch[l + 1])
        b[0] = bias1 if l == 0 else (bias4 if l == 3 else 0.0)
        parts += [W.ravel(), b]
    return np.concatenate(parts)


def test_conv_bf16_emulation_rounds_input_and_activations():
    # one cell, input channel 0 = 0.1874, bias +20 in layer 1 and -20 in
    # the linear layer 4; GELU(x) = x exactly for x >= 20 in FP64 (erf = 1).
    #  FP64: out = (0.1874 + 20) - 20.
    #  BF16: input -> 0.1875 (spacing 2^-10 on [1/8, 1/4)); 20.1875 is a tie
    #        between 20.125 (odd) and 20.25 (even) on the 2^-3 grid above
    #        16 -> 20.25; layers 2-3 keep 20.25; out = 0.25.
    #        (Without the input rounding: 20.1874 -> 20.125, out 0.125;
    #        without the activation rounding: out 0.1875.)
    prm = _delta_net(20.0, -20.0)
    inp = np.array([0.1874, 0.0, 0.0, 0.0])
    o64 = oracle.conv_forward((1, 1, 1), prm, inp)
    obf = oracle.conv_forward((1, 1, 1), prm, inp, bf16=True)
    assert o64.tolist() == [(0.1874 + 20.0) - 20.0, 0.0, 0.0]
    assert obf.tolist() == [0.25, 0.0, 0.0]


def test_conv_bf16_emulation_rounds_weights():
    # input 0 and bias +20 give activations of exactly 20 in layers 1-3;
    # the linear layer's centre weight 1 + 2^-9 rounds to 1 in bfloat16, so
    # the emulated output is -20 + 20 = 0 and the FP64 one 20 * 2^-9
    prm = _delta_net(20.0, -20.0)
    ch = oracle.CONV_CH
    off4 = sum(ch[l + 1] * ch[l] * 27 + ch[l + 1] for l in range(3))
    prm[off4 + 13] = 1.0 + 2.0 ** -9           # layer-4 centre tap, (0, 0)
    inp = np.zeros(4)
    assert oracle.conv_forward((1, 1, 1), prm, inp).tolist()[0] == 20.0 * 2.0 ** -9
    assert oracle.conv_forward((1, 1, 1), prm, inp, bf16=True).tolist()[0] == 0.0
