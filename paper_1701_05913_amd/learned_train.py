"""Train the learned preconditioner stage on the GPU and evaluate it.

Harvest (default, "arnoldi"): for each training system (seeded black-oil
generator), FGMRES(30)+BILU(0) runs three restart cycles from x = 0; a
seeded subset of the cycles' Krylov basis vectors v_j (the vectors the
stage is applied to inside FGMRES) gives inputs r1 = v_j - A z1 with
z1 = BILU(0)^-1 v_j.  Trained with the residual loss, which needs no
target.  ("residual": after every cycle the current residual v = b - A x
gives r1 and its exact target A^-1 r1 = (x_true - x) - z1.)  Each input is
normalised by s = ||r1|| / sqrt(n) (LearnedMakePair) and kept in device
memory.

Train: Adam, one pair per step, cosine learning-rate decay, seeded
shuffling, on one of two losses:
  mse       mean squared error of the output against the normalised
            target A^-1 r1 / s;
  residual  ||A e - r1 / s||^2 / n for the output e (what the stage's
            acceptance test measures; its gradient (2/n) A^T (A e - r1/s)
            needs A and its transpose, kept on the device per system).
The checkpoint (parameters, Adam moments, step count) is written with
LearnedSave; --init starts from the parameters of a checkpoint.

Evaluate: FGMRES(30) with BILU(0) alone and with the learned stage on
held-out seeds, to the same relative tolerance; iterations, wall time and
the fraction of stage applications that fell back.

Every arithmetic step runs in libkrylov.so; torch only provides device
memory.

  python -m paper_1701_05913_amd.learned_train --out weights.bin
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np
import torch

import paper_1701_05913_amd as K
import reservoir_inputs as ri

DEV = "cuda:0"


# base preconditioners of the stage: (plain kind, learned kind)
BASES = {"bilu0": (K.KRY_PC_BILU0, K.KRY_PC_BILU0_LEARNED),
         "cpr_f32": (K.KRY_PC_CPR, K.KRY_PC_CPR_LEARNED)}


class System:
    """One generated system uploaded through the C ABI."""

    def __init__(self, grid, seed, perm="layered", transpose=False):
        # layered fields with variance 2, channelized ones with variance 3
        s = ri.blackoil_system(*grid, seed=seed, perm=perm,
                               sigma2=3.0 if perm == "channelized" else 2.0)
        self.grid, self.seed = grid, seed
        self.nb, self.n = s["nb"], s["n"]
        self.map = K.MapCreateLocal(self.n)
        self.A = K.MatCreateBSR(self.map, self.nb, 3, np.asarray(s["rowptr"], np.int32),
                                np.asarray(s["col"], np.int32),
                                np.ascontiguousarray(np.asarray(s["val"], np.float64).reshape(-1)))
        self.b = torch.from_numpy(np.asarray(s["b"], np.float64)).to(DEV)
        self.x_true = torch.from_numpy(np.asarray(s["x_true"], np.float64)).to(DEV)
        self.lnk = torch.from_numpy(np.asarray(s["lnk"], np.float32)).to(DEV)
        self.At = None
        if transpose:
            # the generator shares one block between A_ij and A_ji, so A^T has
            # A's pattern with every block transposed in place
            tv = np.ascontiguousarray(np.asarray(s["val"], np.float64).reshape(-1, 3, 3)
                                      .transpose(0, 2, 1).reshape(-1))
            self.At = K.MatCreateBSR(self.map, self.nb, 3, np.asarray(s["rowptr"], np.int32),
                                     np.asarray(s["col"], np.int32), tv)
        self._vecs = []

    def vec(self, t):
        h = K.VecWrap(self.map, t)
        self._vecs.append(h)
        return h

    def solver(self, pc, restart=30, rtol=1e-8, maxit=2000, params=None, base="bilu0"):
        """FGMRES with the base preconditioner `base` (BASES), plain (pc =
        its plain kind) or with the learned stage (its learned kind)."""
        S = K.SolverCreate(K.KRY_FGMRES, pc, self.map)
        K.SolverSetMat(S, self.A)
        K.SolverSetStream(S, torch.cuda.current_stream())
        if base == "cpr_f32":
            K.SolverSetPrecision(S, K.KRY_PREC_F32)
            K.SolverSetCPR(S, K.KRY_CPR_PF, 4)
        K.SolverSetRestart(S, restart)
        K.SolverSetRtol(S, rtol)
        K.SolverSetMaxit(S, maxit)
        if params is not None:
            K.SolverSetLearnedParams(S, np.ascontiguousarray(params, np.float32), self.lnk)
        K.SolverAssemble(S)
        return S

    def close(self):
        torch.cuda.synchronize()
        for h in self._vecs:
            K.VecDestroy(h)
        if self.At is not None:
            K.MatDestroy(self.At)
        K.MatDestroy(self.A)
        K.MapDestroy(self.map)


def harvest(sys_, restart, cycles, stop_relres=1e-10):
    """Pairs (input, target) on the device from restart cycles of one solve."""
    K.KrylovSetStream(torch.cuda.current_stream())
    S = sys_.solver(K.KRY_PC_BILU0, restart=restart, rtol=0.0, maxit=restart)
    n, cells = sys_.n, sys_.nb
    x = torch.zeros(n, dtype=torch.float64, device=DEV)
    v = torch.empty_like(x)
    z1 = torch.empty_like(x)
    r1 = torch.empty_like(x)
    d = torch.empty_like(x)
    hb, hx, hv, hz, hr, hd = (sys_.vec(t) for t in (sys_.b, x, v, z1, r1, d))
    hxt = sys_.vec(sys_.x_true)
    bnorm = K.VecNorm2(hb)
    pairs = []
    for _ in range(cycles):
        K.SolverSolve(S, hb, hx)                     # one FGMRES(m) cycle from x
        v.copy_(sys_.b)
        K.MatVecAMXPBY(-1.0, sys_.A, hx, 1.0, hv)    # v = b - A x
        if K.VecNorm2(hv) <= stop_relres * bnorm:
            break
        K.SolverPCApply(S, hv, hz)                   # z1 = BILU(0)^-1 v
        r1.copy_(v)
        K.MatVecAMXPBY(-1.0, sys_.A, hz, 1.0, hr)    # r1 = v - A z1
        K.VecAXPBYZ(1.0, hxt, -1.0, hx, hd)          # d = x_true - x
        K.VecAXPBY(-1.0, hz, 1.0, hd)                # d -= z1  (= A^-1 r1)
        inp = torch.empty(4 * cells, dtype=torch.float32, device=DEV)
        tgt = torch.empty(3 * cells, dtype=torch.float32, device=DEV)
        K.LearnedMakePair(cells, r1, d, sys_.lnk, inp, tgt)
        pairs.append((inp, tgt))
    K.SolverDestroy(S)
    return pairs


def harvest_arnoldi(sys_, npairs, seed, restart=30, cycles=3, base="bilu0"):
    """Stage inputs from the vectors the stage is applied to: the Krylov
    basis vectors v_j of FGMRES(restart) cycles from x = 0 with the base
    preconditioner M, each turned into r1 = v_j - A M^-1 v_j (the residual
    loss needs no target).  A seeded subset of npairs of the cycles'
    vectors is kept."""
    K.KrylovSetStream(torch.cuda.current_stream())
    S = sys_.solver(BASES[base][0], restart=restart, rtol=0.0, maxit=restart, base=base)
    n, cells = sys_.n, sys_.nb
    x = torch.zeros(n, dtype=torch.float64, device=DEV)
    v = torch.empty_like(x)
    z1 = torch.empty_like(x)
    r1 = torch.empty_like(x)
    zero = torch.zeros_like(x)
    hb, hx, hv, hz, hr = (sys_.vec(t) for t in (sys_.b, x, v, z1, r1))
    rng = np.random.default_rng(seed)
    cand = [(c, j) for c in range(cycles) for j in range(1, restart + 1)]
    keep = set(map(tuple, np.array(cand)[rng.choice(len(cand), min(npairs, len(cand)), replace=False)]))
    tgt = torch.zeros(3 * cells, dtype=torch.float32, device=DEV)   # unused by the residual loss
    pairs = []
    for c in range(cycles):
        K.SolverSolve(S, hb, hx)                     # one FGMRES cycle from x
        cols = [j for j in range(1, restart + 1) if (c, j) in keep]
        if not cols:
            continue
        for j in cols:
            K.SolverGetKrylovBasis(S, j, 1, n, out=v)
            K.SolverPCApply(S, hv, hz)               # z1 = M^-1 v_j_j
            r1.copy_(v)
            K.MatVecAMXPBY(-1.0, sys_.A, hz, 1.0, hr)    # r1 = v_j - A z1
            inp = torch.empty(4 * cells, dtype=torch.float32, device=DEV)
            K.LearnedMakePair(cells, r1, zero, sys_.lnk, inp, tgt)
            pairs.append((inp, tgt))
    K.SolverDestroy(S)
    return pairs


def init_params(seed, last_scale=0.1):
    """Uniform(-1/sqrt(fan_in), +1/sqrt(fan_in)); the output layer scaled
    down so the first corrections are small."""
    rng = np.random.default_rng(seed)
    ch = (4, 32, 32, 32, 3)
    out = []
    for l in range(4):
        fan = ch[l] * 27
        bound = 1.0 / math.sqrt(fan)
        sc = last_scale if l == 3 else 1.0
        out.append(sc * rng.uniform(-bound, bound, ch[l + 1] * fan))
        out.append(sc * rng.uniform(-bound, bound, ch[l + 1]))
    return np.concatenate(out).astype(np.float32)


def zero_loss(pairs, grid, loss):
    """Mean loss of the zero network: the mean square of the targets (mse)
    or 1 (residual, by the normalisation)."""
    if loss == "residual":
        return 1.0
    L = K.LearnedCreate(*grid, True)
    K.LearnedSetStream(L, torch.cuda.current_stream())
    K.LearnedSetParams(L, np.zeros(K.LearnedNumParams(), np.float32))
    tot = sum(K.LearnedLossGrad(L, inp, tgt) for inp, tgt, _ in pairs)
    K.LearnedDestroy(L)
    return tot / max(len(pairs), 1)


def train(pairs, grid, epochs, lr, seed, loss="mse", systems=None, init=None, log_every=500,
          save_path=None, resume=None, start_epoch=0, last_scale=0.1):
    """pairs: (input, target, system index); systems: needed for the
    residual loss.  save_path: checkpoint written after every epoch.
    resume, start_epoch: continue a run from the checkpoint it wrote after
    epoch start_epoch - 1 (parameters, Adam moments and step count), with
    the same shuffles and learning-rate schedule as an uninterrupted run."""
    L = K.LearnedCreate(*grid, True)
    K.LearnedSetStream(L, torch.cuda.current_stream())
    if resume is not None:
        K.LearnedLoad(L, resume)
    else:
        K.LearnedSetParams(L, init_params(seed, last_scale) if init is None else init)
    cells = grid[0] * grid[1] * grid[2]
    out = torch.empty(3 * cells, dtype=torch.float32, device=DEV)
    dout = torch.empty_like(out)
    rng = np.random.default_rng(seed)
    total = epochs * len(pairs)
    step, curve, t0 = 0, [], time.perf_counter()
    for ep in range(epochs):
        order = rng.permutation(len(pairs))
        if ep < start_epoch:
            step += len(pairs)
            continue
        acc = 0.0
        for i in order:
            inp, tgt, k = pairs[i]
            if loss == "mse":
                lv = K.LearnedLossGrad(L, inp, tgt)
            else:
                K.LearnedForward(L, inp, out)
                lv = K.LearnedResidualGrad(L, systems[k].A, systems[k].At, inp, out, dout)
                K.LearnedBackward(L, dout)
            lr_t = 0.5 * lr * (1.0 + math.cos(math.pi * step / max(total, 1)))
            K.LearnedAdamStep(L, lr_t, 0.9, 0.999, 1e-8)
            acc += lv
            step += 1
            if step % log_every == 0:
                print(f"  step {step}/{total} loss {lv:.4e}", flush=True)
        curve.append(acc / len(pairs))
        print(f"epoch {ep}: mean loss {curve[-1]:.4e} ({time.perf_counter() - t0:.1f} s)", flush=True)
        if save_path:
            K.LearnedSave(L, save_path)
    return L, curve, time.perf_counter() - t0


def evaluate(grid, seeds, params, rtol=1e-8, restart=30, perm="layered", base="bilu0"):
    rows = []
    for seed in seeds:
        sys_ = System(grid, seed, perm=perm)
        row = {"seed": seed, "grid": list(grid), "perm": perm, "base": base}
        for name, pc, prm in [(base, BASES[base][0], None),
                              (base + "_learned", BASES[base][1], params)]:
            S = sys_.solver(pc, restart=restart, rtol=rtol, params=prm, base=base)
            x = torch.zeros(sys_.n, dtype=torch.float64, device=DEV)
            hb, hx = sys_.vec(sys_.b), sys_.vec(x)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc = K.SolverSolve(S, hb, hx)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            ent = {"status": rc, "iters": K.SolverGetIters(S), "relres": K.SolverGetResidual(S),
                   "solve_s": round(dt, 4)}
            if prm is not None:
                a, f = K.SolverGetLearnedStats(S)
                ent["stage_applies"], ent["stage_fallbacks"] = a, f
            row[name] = ent
            K.SolverDestroy(S)
        print(json.dumps(row), flush=True)
        rows.append(row)
        sys_.close()
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", required=True, help="checkpoint file to write")
    ap.add_argument("--grid", default="64,64,64")
    ap.add_argument("--train-seeds", default="0:32", help="first:last (exclusive)")
    ap.add_argument("--eval-seeds", default="10000:10004")
    ap.add_argument("--eval-grids", default="64,64,64;128,128,64",
                    help="grids of the held-out systems, ';'-separated")
    ap.add_argument("--harvest", choices=("arnoldi", "residual"), default="arnoldi",
                    help="stage inputs from FGMRES(30) basis vectors (residual loss only) or "
                         "from restart-cycle residuals with exact targets")
    ap.add_argument("--pairs-per-system", type=int, default=78)
    ap.add_argument("--restart", type=int, default=10, help="FGMRES restart during harvest")
    ap.add_argument("--cycles", type=int, default=40, help="restart cycles harvested per system")
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--last-scale", type=float, default=0.1,
                    help="scale of the output layer's initial weights (0: the first "
                         "corrections are zero)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--loss", choices=("mse", "residual"), default="residual")
    ap.add_argument("--init", default=None, help="checkpoint to start from")
    ap.add_argument("--resume", default=None,
                    help="checkpoint this run wrote after epoch --start-epoch - 1")
    ap.add_argument("--start-epoch", type=int, default=0)
    ap.add_argument("--grid-perm", default="layered", choices=("layered", "channelized"),
                    help="permeability field of the training and evaluation systems")
    ap.add_argument("--base", default="bilu0", choices=sorted(BASES),
                    help="base preconditioner the stage corrects (harvest and evaluation)")
    ap.add_argument("--report", default=None, help="JSON summary file")
    ap.add_argument("--eval-only", action="store_true",
                    help="no harvest or training: evaluate the checkpoint given by --init")
    a = ap.parse_args(argv)
    # torch's CUDA context first, then the library (see the binding's notes)
    torch.zeros(1, device=DEV)
    grid = tuple(int(v) for v in a.grid.split(","))
    t0, t1 = (int(v) for v in a.train_seeds.split(":"))
    e0, e1 = (int(v) for v in a.eval_seeds.split(":"))

    if a.eval_only:
        if not a.init:
            ap.error("--eval-only needs --init")
        Li = K.LearnedCreate(*grid, False)
        K.LearnedLoad(Li, a.init)
        params = K.LearnedGetParams(Li)
        K.LearnedDestroy(Li)
        rows = []
        for eg in a.eval_grids.split(";"):
            rows += evaluate(tuple(int(v) for v in eg.split(",")), range(e0, e1), params,
                         perm=a.grid_perm, base=a.base)
        summary = {"checkpoint": a.init, "eval_seeds": [e0, e1], "eval": rows}
        if a.report:
            with open(a.report, "w") as f:
                json.dump(summary, f, indent=1)
        return
    keep = a.loss == "residual"
    pairs, systems, th = [], [], time.perf_counter()
    if a.harvest == "arnoldi" and a.loss != "residual":
        ap.error("--harvest arnoldi has no targets: use --loss residual")
    if a.harvest == "residual" and a.base != "bilu0":
        ap.error("--harvest residual supports --base bilu0 only")
    for seed in range(t0, t1):
        sys_ = System(grid, seed, perm=a.grid_perm, transpose=keep)
        if a.harvest == "arnoldi":
            p = harvest_arnoldi(sys_, a.pairs_per_system, seed, base=a.base)
        else:
            p = harvest(sys_, a.restart, a.cycles)
        pairs += [(inp, tgt, len(systems)) for inp, tgt in p]
        if keep:
            systems.append(sys_)
        else:
            sys_.close()
        print(f"harvest seed {seed}: {len(p)} pairs (total {len(pairs)})", flush=True)
    t_harvest = time.perf_counter() - th

    init = None
    if a.init:
        Li = K.LearnedCreate(*grid, False)
        K.LearnedLoad(Li, a.init)
        init = K.LearnedGetParams(Li)
        K.LearnedDestroy(Li)
    loss0 = zero_loss(pairs, grid, a.loss)
    print(f"zero-network {a.loss} loss {loss0:.4e} over {len(pairs)} pairs", flush=True)
    if a.resume and not a.start_epoch:
        ap.error("--resume needs --start-epoch")
    L, curve, t_train = train(pairs, grid, a.epochs, a.lr, a.seed, loss=a.loss, systems=systems,
                              init=init, save_path=a.out, resume=a.resume,
                              start_epoch=a.start_epoch, last_scale=a.last_scale)
    params = K.LearnedGetParams(L)
    K.LearnedDestroy(L)
    npairs = len(pairs)
    del pairs
    for sys_ in systems:
        sys_.close()
    torch.cuda.empty_cache()

    rows = []
    for eg in a.eval_grids.split(";"):
        rows += evaluate(tuple(int(v) for v in eg.split(",")), range(e0, e1), params,
                         perm=a.grid_perm, base=a.base)
    summary = {"grid": list(grid), "train_seeds": [t0, t1], "eval_seeds": [e0, e1],
               "harvest": a.harvest, "pairs_per_system": a.pairs_per_system,
               "restart_harvest": a.restart, "cycles": a.cycles, "epochs": a.epochs, "lr": a.lr,
               "loss": a.loss, "init": a.init, "perm": a.grid_perm, "base": a.base,
               "last_scale": a.last_scale,
               "resume": a.resume, "start_epoch": a.start_epoch, "pairs": npairs, "harvest_s": round(t_harvest, 1),
               "train_s": round(t_train, 1), "zero_network_loss": loss0,
               "loss_per_epoch": curve, "eval": rows}
    if a.report:
        with open(a.report, "w") as f:
            json.dump(summary, f, indent=1)
    print(json.dumps({k: v for k, v in summary.items() if k != "eval"}))


if __name__ == "__main__":
    main()
