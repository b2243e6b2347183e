"""Helpers for the GPU tests: upload a generated system through the C ABI
and run one solve.  Marshalling only; the solver runs in libkrylov.so."""
import numpy as np
import torch

import paper_1701_05913_amd as K

DEV = "cuda:0"


class GpuSystem:
    def __init__(self, s, where="host"):
        self.s = s
        self.bs = int(s.get("bs", 1))
        self.nb = len(s["rowptr"]) - 1
        self.n = self.nb * self.bs
        self.map = K.MapCreateLocal(self.n)
        rp = np.ascontiguousarray(s["rowptr"], dtype=np.int32)
        ci = np.ascontiguousarray(s["col"], dtype=np.int32)
        va = np.ascontiguousarray(np.asarray(s["val"], dtype=np.float64).reshape(-1))
        if where == "device":
            rp, ci, va = (torch.from_numpy(a).to(DEV) for a in (rp, ci, va))
        if self.bs == 1:
            self.A = K.MatCreateCSR(self.map, self.nb, rp, ci, va)
        else:
            self.A = K.MatCreateBSR(self.map, self.nb, self.bs, rp, ci, va)
        self._vecs = []

    def vec(self, arr=None):
        t = torch.zeros(self.n, dtype=torch.float64, device=DEV) if arr is None else \
            torch.from_numpy(np.ascontiguousarray(arr, dtype=np.float64)).to(DEV)
        h = K.VecWrap(self.map, t)
        self._vecs.append(h)
        return t, h

    def close(self):
        torch.cuda.synchronize()
        for h in self._vecs:
            K.VecDestroy(h)
        self._vecs = []
        K.MatDestroy(self.A)
        K.MapDestroy(self.map)


def make_solver(g, solver, pc, rtol=1e-8, maxit=5000, restart=30, atol=0.0,
                prec=K.KRY_PREC_F64, cpr=(K.KRY_CPR_PF, 4), layout=K.KRY_SWEEP_AUTO, aug_k=0,
                ras=(4, 1), amg=(8, 2, 4), cpr_p=K.KRY_CPR_P_ILU0, cpr_f=K.KRY_CPR_F_BILU0,
                ortho=K.KRY_ORTHO_AUTO):
    S = K.SolverCreate(solver, pc, g.map)
    K.SolverSetSweepLayout(S, layout)
    K.SolverSetOrthog(S, ortho)
    K.SolverSetMat(S, g.A)
    K.SolverSetRtol(S, rtol)
    K.SolverSetAtol(S, atol)
    K.SolverSetMaxit(S, maxit)
    K.SolverSetRestart(S, restart)
    K.SolverSetAugk(S, aug_k)
    K.SolverSetPrecision(S, prec)
    if pc == K.KRY_PC_CPR:
        K.SolverSetCPR(S, cpr[0], cpr[1])
        K.SolverSetCPRPressure(S, cpr_p)
        K.SolverSetCPRFull(S, cpr_f)
    # (max_levels, num_sweeps, gs_chunk) of AMG, for KRY_PC_AMG and CPR-AMG
    K.SolverSetAMG(S, *amg)
    if pc == K.KRY_PC_RAS or cpr_f == K.KRY_CPR_F_RAS:
        # (nsub, overlap): z-slabs; (px, py, pz, overlap): boxes
        if len(ras) == 4:
            K.SolverSetRASBoxes(S, *ras)
        else:
            K.SolverSetRAS(S, *ras)
    K.SolverSetStream(S, torch.cuda.current_stream())
    return S


def solve(g, solver, pc, b=None, x0=None, **kw):
    S = make_solver(g, solver, pc, **kw)
    try:
        K.SolverAssemble(S)
        bt, bh = g.vec(g.s["b"] if b is None else b)
        xt, xh = g.vec(x0)
        rc = K.SolverSolve(S, bh, xh)
        torch.cuda.synchronize()
        return dict(status=rc, x=xt.cpu().numpy(), iters=K.SolverGetIters(S),
                    relres=K.SolverGetResidual(S), hist=K.SolverGetHistory(S),
                    times=K.SolverGetTimes(S))
    finally:
        K.SolverDestroy(S)


def pc_apply(g, pc, v, prec=K.KRY_PREC_F64, cpr=(K.KRY_CPR_PF, 4), solver=K.KRY_FGMRES,
             layout=K.KRY_SWEEP_AUTO, repeat=1, ras=(4, 1), amg=(8, 2, 4), cpr_p=K.KRY_CPR_P_ILU0,
             cpr_f=K.KRY_CPR_F_BILU0):
    S = make_solver(g, solver, pc, prec=prec, cpr=cpr, layout=layout, ras=ras, amg=amg,
                    cpr_p=cpr_p, cpr_f=cpr_f)
    try:
        K.SolverAssemble(S)
        vt, vh = g.vec(v)
        zt, zh = g.vec()
        outs = []
        for _ in range(repeat):
            K.SolverPCApply(S, vh, zh)
            torch.cuda.synchronize()
            outs.append(zt.cpu().numpy())
        return outs[0] if repeat == 1 else outs
    finally:
        K.SolverDestroy(S)


def relerr(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / (nb if nb > 0 else 1.0)
