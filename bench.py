"""Benchmark: time to a true FP64 relative residual of 1e-8 on one GPU's
share at production scale (the 256x256x128 channelized black-oil system,
25.2 M unknowns), plain FP64 GMRES(30) + block ILU(0) against the
mixed-precision, CPR and learned variants, with the dominant kernel's HBM
roofline and the CPU oracle timed on the host.

One step = one time-to-solution of the headline configuration (plain FP64
GMRES(30) + BILU(0): preconditioner setup + solve from x0 = 0, inputs
resident in HBM).  `value` is the mean over the timed steps.  The variants
(FP32 / BF16-factor FGMRES, FP32 CPR, CPR-FPF, the learned stage) each run
once after the timed region, and one more headline solve with every
instrumented kernel bracketed by HIP events gives the per-kernel table.

    python bench.py [--steps K] [--warmup W] [--workload NAME]
                    [--variants default|all|none|name,...] [--no-cpu]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("time-to-1e-8 residual (s) + iters, plain vs mixed/learned; "
          "SpMV HBM GB/s")
HBM_PEAK_GBS = 8000.0
INFINITY_CACHE_BYTES = 256 << 20

WORKLOADS = {
    "channelized256x256x128": dict(
        grid=(256, 256, 128), perm="channelized", sigma2=3.0, maxit=10000,
        desc="256x256x128 3x3-block black-oil system (25,165,824 unknowns, 58,458,112 "
             "blocks), channelized log-normal permeability (ln k ~ N(0,3), 20% channels "
             "at 1000x), seed 0"),
    "blackoil128x128x64": dict(
        grid=(128, 128, 64), perm="layered", sigma2=2.0, maxit=5000,
        desc="128x128x64 3x3-block black-oil system (3,145,728 unknowns), layered "
             "log-normal permeability, seed 0"),
    "blackoil64": dict(
        grid=(64, 64, 64), perm="layered", sigma2=2.0, maxit=5000,
        desc="64x64x64 3x3-block black-oil system (786,432 unknowns, 1,810,432 blocks), "
             "layered log-normal permeability, seed 0"),
    "blackoil32": dict(grid=(32, 32, 32), perm="layered", sigma2=2.0, maxit=5000,
                       desc="32^3 3x3-block black-oil system (quick check)"),
}

# name, solver, pc, precision, cpr (variant, sweeps)
CONFIGS = [
    ("gmres30_bilu0_f64", "GMRES", "BILU0", "F64", None),
    ("bicgstab_bilu0_f64", "BICGSTAB", "BILU0", "F64", None),
    ("fgmres30_bilu0_f32", "FGMRES", "BILU0", "F32", None),
    ("fgmres30_bilu0_bf16", "FGMRES", "BILU0", "BF16_FACTORS", None),
    ("fgmres30_cpr_f64", "FGMRES", "CPR", "F64", ("PF", 4)),
    ("fgmres30_cpr_f32", "FGMRES", "CPR", "F32", ("PF", 4)),
    ("fgmres30_cpr_bf16", "FGMRES", "CPR", "BF16_FACTORS", ("PF", 4)),
    ("fgmres30_cpr_fpf_f64", "FGMRES", "CPR", "F64", ("FPF", 4)),
    ("fgmres30_cpr_ffpf_f64", "FGMRES", "CPR", "F64", ("FFPF", 4)),
    ("fgmres30_bilu0_learned", "FGMRES", "BILU0_LEARNED", "F64", None),
    ("fgmres30_bilu0_f64_heldout", "FGMRES", "BILU0", "F64", None),
    ("fgmres30_cpr_f32_learned", "FGMRES", "CPR_LEARNED", "F32", ("PF", 4)),
    ("fgmres30_cpr_f32_heldout", "FGMRES", "CPR", "F32", ("PF", 4)),
    ("lgmres30_2_bilu0_f64", "GMRES", "BILU0", "F64", None),
    ("pcg_ilu0_scalar_f64", "CG", "ILU0", "F64", None),
    ("gmres30_ras4_f64", "GMRES", "RAS", "F64", None),
    ("gmres30_ras8_f64", "GMRES", "RAS", "F64", None),
    ("gmres30_rasbox_1x4x4_f64", "GMRES", "RAS", "F64", None),
    ("gmres30_rasbox_2x4x4_f64", "GMRES", "RAS", "F64", None),
    ("gmres30_rasbox_2x2x2_f64", "GMRES", "RAS", "F64", None),
    ("gmres30_ilu0_scalar_f64", "GMRES", "ILU0", "F64", None),
    ("gmres30_amg_scalar_f64", "GMRES", "AMG", "F64", None),
    ("fgmres30_cpr_fpf_amg_f64", "FGMRES", "CPR", "F64", ("FPF", 4)),
    ("fgmres30_cpr_fpf_ras_f64", "FGMRES", "CPR", "F64", ("FPF", 4)),
    ("fgmres30_cpr_fpf_ras_amg_f64", "FGMRES", "CPR", "F64", ("FPF", 4)),
]
# per-configuration extras: LGMRES augmentation, and the symmetric scalar
# system of the same grid (CG needs a symmetric positive definite matrix)
# The learned variants run on a system of the same workload drawn with a seed
# that no training run used (HELDOUT_SEED), each beside the same solve
# without the stage (the *_heldout rows).
EXTRAS = {"lgmres30_2_bilu0_f64": dict(aug_k=2), "pcg_ilu0_scalar_f64": dict(system="scalar"),
          "fgmres30_bilu0_learned": dict(system="heldout"),
          "fgmres30_bilu0_f64_heldout": dict(system="heldout"),
          "fgmres30_cpr_f32_learned": dict(system="heldout", weights="cpr_f32_channelized128.bin"),
          "fgmres30_cpr_f32_heldout": dict(system="heldout"),
          "gmres30_ras4_f64": dict(ras=(4, 1)), "gmres30_ras8_f64": dict(ras=(8, 1)),
          "gmres30_rasbox_1x4x4_f64": dict(ras=(1, 4, 4, 1)),
          "gmres30_rasbox_2x4x4_f64": dict(ras=(2, 4, 4, 1)),
          "gmres30_rasbox_2x2x2_f64": dict(ras=(2, 2, 2, 1)),
          "gmres30_ilu0_scalar_f64": dict(system="scalar"),
          "gmres30_amg_scalar_f64": dict(system="scalar"),
          "fgmres30_cpr_fpf_amg_f64": dict(cpr_pressure="AMG"),
          # the paper's CPR: full stage R(A)^-1 = RAS (1x4x4 boxes, overlap 1)
          "fgmres30_cpr_fpf_ras_f64": dict(cpr_full="RAS", ras=(1, 4, 4, 1)),
          "fgmres30_cpr_fpf_ras_amg_f64": dict(cpr_full="RAS", ras=(1, 4, 4, 1),
                                               cpr_pressure="AMG")}
HEADLINE = "gmres30_bilu0_f64"
# variants run once after the timed region unless --variants says otherwise
DEFAULT_VARIANTS = {
    "channelized256x256x128": ["fgmres30_bilu0_f32", "fgmres30_bilu0_bf16", "fgmres30_cpr_f32",
                               "fgmres30_cpr_fpf_f64", "fgmres30_cpr_f32_heldout",
                               "fgmres30_cpr_f32_learned"],
    "blackoil128x128x64": ["fgmres30_bilu0_f32", "fgmres30_bilu0_bf16", "fgmres30_cpr_f64",
                           "fgmres30_cpr_f32", "fgmres30_cpr_bf16", "fgmres30_cpr_fpf_f64"],
    "blackoil64": [c[0] for c in CONFIGS if c[0] != HEADLINE],
    "blackoil32": ["fgmres30_bilu0_f32"],
}
WEIGHTS_DIR = os.path.join(ROOT, "paper_1701_05913_amd", "weights")
WEIGHTS = "bilu0_blackoil64.bin"
HELDOUT_SEED = 10000

# matrix-core FLOPs per cell of each conv layer (3x3x3 taps, 2 per MAC)
CONV_FLOPS_PER_CELL = {"conv_l1_fwd": 2 * 27 * 4 * 32, "conv_l2_fwd": 2 * 27 * 32 * 32,
                       "conv_l3_fwd": 2 * 27 * 32 * 32, "conv_l4_fwd": 2 * 27 * 32 * 3}
MFMA_BF16_PEAK_TFLOPS = 2500.0
# the kernels whose launches the timed region brackets with HIP events (one
# launch in ROOF_SAMPLE): the headline's candidates for the dominant kernel
ROOF_CANDIDATES = ("ilu_bwd_bsr3_f64", "ilu_fwd_bsr3_f64", "spmv_bsr3")
ROOF_SAMPLE = 8
RESTART = 30


def algorithmic_bytes(nb, nnzb):
    """Minimum HBM bytes per launch of each timed kernel family (each matrix
    byte once, each vector once): 3x3 blocks with int32 column indices."""
    nl = (nnzb - nb) // 2          # strictly lower blocks (= upper) of a 7-point stencil
    ptr = 4 * (nb + 1)
    return {
        "spmv_bsr3": 76 * nnzb + ptr + 48 * nb,
        "ilu_fwd_bsr3_f64": 76 * nl + ptr + 48 * nb,
        "ilu_bwd_bsr3_f64": 76 * nl + 72 * nb + ptr + 48 * nb,
        # FP32 factors: 40 B per block, FP32 intermediate, FP64 in/out
        "ilu_fwd_bsr3_f32": 40 * nl + ptr + 24 * nb + 12 * nb,
        "ilu_bwd_bsr3_f32": 40 * nl + 36 * nb + ptr + 12 * nb + 24 * nb,
        # BF16 factors: 22 B per block, FP32 diagonal inverses
        "ilu_fwd_bsr3_bf16": 22 * nl + ptr + 24 * nb + 12 * nb,
        "ilu_bwd_bsr3_bf16": 22 * nl + 36 * nb + ptr + 12 * nb + 24 * nb,
        # CPR second stage: the backward sweep also reads the pressure
        # correction (one value per cell) and writes the combined FP64 result
        "ilu_bwd_bsr3_f64_inject": 76 * nl + 72 * nb + ptr + 48 * nb + 8 * nb + 24 * nb,
        "ilu_bwd_bsr3_f32_inject": 40 * nl + 36 * nb + ptr + 12 * nb + 12 * nb + 4 * nb + 24 * nb,
    }


def cgs2_step_bytes(n, nc):
    """Algorithmic bytes of one CGS2 Arnoldi step against nc basis columns:
    pass 1 reads V and w, pass 2 reads V and w and writes w (its norm
    fused), pass 3 reads V and w and writes the next basis vector (the
    scaling fused): (3 nc + 5) n doubles."""
    return (3 * nc + 5) * n * 8


def dcgs2_step_bytes(n, nc):
    """Algorithmic bytes of one step of the lagged CGS2 against nc basis
    columns (the last one the once-projected vector u): pass A reads them
    and w, pass B reads them and w again and writes the final v_j and the
    next once-projected vector (its norm fused): (2 nc + 4) n doubles."""
    return (2 * nc + 4) * n * 8


def cgs2_avg_bytes(n, iters, launches, restart=RESTART, step_bytes=cgs2_step_bytes):
    """Average algorithmic bytes per Arnoldi step (CGS2, or with
    step_bytes=dcgs2_step_bytes the lagged form) over a GMRES(restart)
    solve of `iters` steps; steps issued past the converged one (at most
    one per solve) are counted with the next column count."""
    full, rem = divmod(iters, restart)
    tot = full * sum(step_bytes(n, c) for c in range(1, restart + 1))
    tot += sum(step_bytes(n, c) for c in range(1, rem + 1))
    extra = max(0, launches - iters)
    tot += extra * step_bytes(n, min(rem + 1, restart))
    return tot / max(1, launches)


def traffic_from_profiles(kernel, workload):
    """HBM bytes per launch measured with rocprofv3 FETCH_SIZE/WRITE_SIZE
    for this kernel on this workload, if a summary exists and the kernel's
    source has not changed since."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        data = json.load(open(path))
        ent = data.get(workload, {}).get(kernel)
        if not ent:
            return None
        src = os.path.join(ROOT, ent["source"])
        h = hashlib.sha256(open(src, "rb").read()).hexdigest()
        if h != ent["source_sha256"]:
            return None
        return float(ent["bytes_per_launch"])
    except Exception:
        return None


def host_cpu():
    model = "unknown"
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return model, avail


def _oracle_leg(oracle, s, rtol, gpu_iters, budget_s, threads):
    """BILU(0) setup + GMRES(30) with the oracle library currently selected:
    the whole solve when a short prefix says it fits the budget, else a
    fixed-iteration prefix that fits, scaled to the GPU's iteration count."""
    A = oracle.Matrix.from_system(s)
    t0 = time.perf_counter()
    pc = oracle.PC(A, "bilu0")
    t_setup = time.perf_counter() - t0
    k0 = 2
    t0 = time.perf_counter()
    oracle.gmres(A, pc, s["b"], restart=RESTART, maxit=k0, rtol=0.0, fixed_iters=True)
    per_it = (time.perf_counter() - t0) / k0
    common = dict(unit="s", cores=threads, kind="oracle")
    if t_setup + per_it * (gpu_iters + RESTART) < budget_s:
        t0 = time.perf_counter()
        r = oracle.gmres(A, pc, s["b"], restart=RESTART, maxit=10000, rtol=rtol)
        t_solve = time.perf_counter() - t0
        return dict(value=round(t_setup + t_solve, 4), iters=r["iters"],
                    true_relres=r["relres"], setup_s=round(t_setup, 3),
                    sample="the whole workload: BILU(0) setup + GMRES(30) solve to the same rtol",
                    **common)
    k = int((budget_s - t_setup) / per_it) - k0
    if k >= 2 * k0:     # a longer prefix, if the budget has room for one
        t0 = time.perf_counter()
        oracle.gmres(A, pc, s["b"], restart=RESTART, maxit=k, rtol=0.0, fixed_iters=True)
        per_it = (time.perf_counter() - t0) / k
    else:
        k = k0
    return dict(value=round(t_setup + per_it * gpu_iters, 2), setup_s=round(t_setup, 3),
                s_per_iter=round(per_it, 4),
                sample=f"BILU(0) setup + a {k}-iteration GMRES(30) prefix timed, scaled to the "
                       f"GPU's {gpu_iters} iterations", **common)


def cpu_baseline(s, rtol, gpu_iters, budget_s=30.0):
    """The FP64 oracle on the host, two legs: the plain build on one thread
    (the correctness reference) and the OpenMP build (parallel SpMV, dot
    products and vector loops, serial sweeps and factorization) over every
    core this process may use.  `value` is the OpenMP leg."""
    import oracle
    model, avail = host_cpu()
    single = _oracle_leg(oracle, s, rtol, gpu_iters, budget_s, 1)
    omp = None
    try:
        lib = oracle.load(oracle.build_omp(force=False))
        threads = int(os.environ.get("OMP_NUM_THREADS", avail))
        with oracle.using(lib):
            omp = _oracle_leg(oracle, s, rtol, gpu_iters, budget_s, threads)
    except Exception as e:          # no OpenMP toolchain: report the single leg
        print(f"[bench] OpenMP oracle leg skipped: {e}", file=sys.stderr)
    out = dict(omp if omp else single)
    out.update(cpu_model=model, nproc=avail, single_thread=single)
    return out


def build_solver(K, name, st, pc, prec, cpr, ex, mm, AA, rtol, maxit, stream, lnk):
    S = K.SolverCreate(getattr(K, f"KRY_{st}"), getattr(K, f"KRY_PC_{pc}"), mm)
    K.SolverSetMat(S, AA)
    K.SolverSetRtol(S, rtol)
    K.SolverSetMaxit(S, maxit)
    K.SolverSetRestart(S, RESTART)
    K.SolverSetAugk(S, ex.get("aug_k", 0))
    if "ras" in ex:   # (nsub, overlap) z-slabs or (px, py, pz, overlap) boxes
        if len(ex["ras"]) == 4:
            K.SolverSetRASBoxes(S, *ex["ras"])
        else:
            K.SolverSetRAS(S, *ex["ras"])
    K.SolverSetPrecision(S, getattr(K, f"KRY_PREC_{prec}"))
    if cpr:
        K.SolverSetCPR(S, getattr(K, f"KRY_CPR_{cpr[0]}"), cpr[1])
        K.SolverSetCPRPressure(S, getattr(K, f"KRY_CPR_P_{ex.get('cpr_pressure', 'ILU0')}"))
        K.SolverSetCPRFull(S, getattr(K, f"KRY_CPR_F_{ex.get('cpr_full', 'BILU0')}"))
    K.SolverSetStream(S, stream)
    if pc.endswith("_LEARNED"):
        K.SolverSetLearned(S, os.path.join(WEIGHTS_DIR, ex.get("weights", WEIGHTS)), lnk)
    return S


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="channelized256x256x128", choices=sorted(WORKLOADS))
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=30.0,
                    help="seconds of oracle work per CPU leg")
    ap.add_argument("--variants", default="default")
    ap.add_argument("--flush", action="store_true",
                    help="write a 512 MiB scratch buffer between timed steps (the working "
                         "set of the smaller workloads fits the 256 MiB Infinity Cache)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run one device-to-device copy of MIB MiB (the reference "
                         "kernel for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE) and exit")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        src = torch.ones(args.copy_probe * 131072, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": src.numel() * 8}))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU holding one rank's share; "
              "multi-GPU runs are not supported (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1701_05913_amd as K
    import reservoir_inputs as ri

    wl = WORKLOADS[args.workload]
    print(f"[bench] generating {args.workload}", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    s = ri.blackoil_system(*wl["grid"], seed=0, perm=wl["perm"], sigma2=wl["sigma2"])
    t_gen = time.perf_counter() - t0
    nb = len(s["rowptr"]) - 1
    n = 3 * nb
    nnzb = int(s["rowptr"][-1])
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    rp = torch.from_numpy(np.ascontiguousarray(s["rowptr"], dtype=np.int32)).to(dev)
    ci = torch.from_numpy(np.ascontiguousarray(s["col"], dtype=np.int32)).to(dev)
    va = torch.from_numpy(np.ascontiguousarray(s["val"].reshape(-1))).to(dev)
    b = torch.from_numpy(s["b"]).to(dev)
    x = torch.zeros(n, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    K.KrylovSetStream(stream)
    m = K.MapCreateLocal(n)
    A = K.MatCreateBSR(m, nb, 3, rp, ci, va)
    torch.cuda.synchronize()
    del rp, ci, va
    t_upload = time.perf_counter() - t0
    print(f"[bench] generated in {t_gen:.1f} s, uploaded in {t_upload:.1f} s",
          file=sys.stderr, flush=True)
    bh, xh = K.VecWrap(m, b), K.VecWrap(m, x)
    lnk = torch.from_numpy(np.asarray(s["lnk"], dtype=np.float32)).to(dev)

    if args.variants == "default":
        vnames = DEFAULT_VARIANTS.get(args.workload, [])
    elif args.variants == "all":
        vnames = [c[0] for c in CONFIGS if c[0] != HEADLINE]
    elif args.variants == "none":
        vnames = []
    else:
        vnames = [v for v in args.variants.split(",") if v]
    known = {c[0]: c for c in CONFIGS}
    for v in vnames:
        if v not in known:
            sys.exit(f"unknown variant {v}")
    configs = [known[HEADLINE]] + [known[v] for v in vnames if v != HEADLINE]

    # the scalar system, built only when a configuration needs it
    sys_vecs = {"blackoil": (m, A, bh, xh, x, lnk)}
    # learned variants without their weights file are skipped
    for c in list(configs):
        w = EXTRAS.get(c[0], {}).get("weights", WEIGHTS)
        if c[2].endswith("_LEARNED") and not os.path.exists(os.path.join(WEIGHTS_DIR, w)):
            print(f"[bench] {c[0]}: no weights file {w}, skipped", file=sys.stderr, flush=True)
            configs.remove(c)
    if any(EXTRAS.get(c[0], {}).get("system") == "heldout" for c in configs):
        sh = ri.blackoil_system(*wl["grid"], seed=HELDOUT_SEED, perm=wl["perm"],
                                sigma2=wl["sigma2"])
        m2 = K.MapCreateLocal(n)
        A2 = K.MatCreateBSR(m2, nb, 3,
                            torch.from_numpy(np.ascontiguousarray(sh["rowptr"], dtype=np.int32)).to(dev),
                            torch.from_numpy(np.ascontiguousarray(sh["col"], dtype=np.int32)).to(dev),
                            torch.from_numpy(np.ascontiguousarray(sh["val"].reshape(-1))).to(dev))
        b2 = torch.from_numpy(sh["b"]).to(dev)
        x2 = torch.zeros(n, dtype=torch.float64, device=dev)
        lnk2 = torch.from_numpy(np.asarray(sh["lnk"], dtype=np.float32)).to(dev)
        sys_vecs["heldout"] = (m2, A2, K.VecWrap(m2, b2), K.VecWrap(m2, x2), x2, lnk2)
        del sh
    if any(EXTRAS.get(c[0], {}).get("system") == "scalar" for c in configs):
        ss = ri.scalar_system(*wl["grid"], seed=0)
        ns = len(ss["rowptr"]) - 1
        m1 = K.MapCreateLocal(ns)
        A1 = K.MatCreateCSR(m1, ns, torch.from_numpy(np.ascontiguousarray(ss["rowptr"], dtype=np.int32)).to(dev),
                            torch.from_numpy(np.ascontiguousarray(ss["col"], dtype=np.int32)).to(dev),
                            torch.from_numpy(np.ascontiguousarray(ss["val"].reshape(-1))).to(dev))
        b1 = torch.from_numpy(ss["b"]).to(dev)
        x1 = torch.zeros(ns, dtype=torch.float64, device=dev)
        sys_vecs["scalar"] = (m1, A1, K.VecWrap(m1, b1), K.VecWrap(m1, x1), x1, None)
    solvers = {}
    for name, st, pc, prec, cpr in configs:
        ex = EXTRAS.get(name, {})
        mm, AA = sys_vecs[ex.get("system", "blackoil")][:2]
        solvers[name] = build_solver(K, name, st, pc, prec, cpr, ex, mm, AA, args.rtol,
                                     wl["maxit"], stream, sys_vecs[ex.get("system", "blackoil")][5])

    flush_buf = None
    if args.flush:
        flush_buf = torch.empty(512 << 17, dtype=torch.float64, device=dev)

    def run_one(name, quiet=False):
        S = solvers[name]
        _, _, bv, xv, xt, _ = sys_vecs[EXTRAS.get(name, {}).get("system", "blackoil")]
        xt.zero_()
        if flush_buf is not None:
            flush_buf.fill_(1.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        K.SolverAssemble(S)
        rc = K.SolverSolve(S, bv, xv)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st, ss_ = K.SolverGetTimes(S)
        out = dict(time_s=dt, setup_s=st, solve_s=ss_, iters=K.SolverGetIters(S),
                   true_relres=K.SolverGetResidual(S), status=rc)
        if name.endswith("_learned"):
            out["stage_applies"], out["stage_fallbacks"] = K.SolverGetLearnedStats(S)
        if not quiet:
            print(f"[bench] {name}: {dt:.4f} s, {out['iters']} iterations, true relres "
                  f"{out['true_relres']:.2e}", file=sys.stderr, flush=True)
        return out

    for _ in range(args.warmup):
        run_one(HEADLINE)

    # timed region: the headline solve; HIP events bracket one launch in
    # every ROOF_SAMPLE of the candidate dominant kernels (every event adds
    # a few microseconds between the launches it separates)
    K.KernelTimingReset()
    K.KernelTimingSelect(",".join(ROOF_CANDIDATES))
    K.KernelTimingSample(ROOF_SAMPLE)
    K.KernelTimingEnable(True)
    results = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        results.append(run_one(HEADLINE))
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    K.KernelTimingEnable(False)
    timed = {k: K.KernelTimingQuery(k) for k in ROOF_CANDIDATES}

    # per-kernel table: one untimed headline solve with every instrumented
    # launch bracketed
    K.KernelTimingReset()
    K.KernelTimingSelect(None)
    K.KernelTimingSample(1)
    K.KernelTimingEnable(True)
    prof = run_one(HEADLINE, quiet=True)
    torch.cuda.synchronize()
    K.KernelTimingEnable(False)
    abytes = algorithmic_bytes(nb, nnzb)
    kernels = {}
    for kname in list(abytes) + ["cgs2", "dcgs2", "ilu_grid_untile",
                                 "ilu_grid_factor", "spmv_csr"]:
        cnt, ms = K.KernelTimingQuery(kname)
        if cnt == 0:
            continue
        ent = dict(launches=cnt, total_ms=round(ms, 4), avg_us=round(1000 * ms / cnt, 3))
        bpl = abytes.get(kname)
        if kname == "cgs2":
            bpl = int(cgs2_avg_bytes(n, prof["iters"], cnt))
        elif kname == "dcgs2":
            bpl = int(cgs2_avg_bytes(n, prof["iters"], cnt, step_bytes=dcgs2_step_bytes))
        if bpl:
            gbs = bpl / (ms / cnt * 1e-3) / 1e9
            ent.update(bytes_per_launch=bpl, gbs=round(gbs, 1), frac_hbm=round(gbs / HBM_PEAK_GBS, 4))
        kernels[kname] = ent
    head_kernels = dict(kernels)

    # variants: each once, untimed, every instrumented launch bracketed
    variants = {}
    K.KernelTimingReset()
    K.KernelTimingEnable(True)
    for name, *_ in configs[1:]:
        r = run_one(name)
        variants[name] = dict(time_s=round(r["time_s"], 5), setup_s=round(r["setup_s"], 5),
                              solve_s=round(r["solve_s"], 5), iters=r["iters"],
                              true_relres=r["true_relres"], converged=r["status"] == 0)
        if "stage_applies" in r:
            variants[name].update(stage_applies=r["stage_applies"],
                                  stage_fallbacks=r["stage_fallbacks"])
    torch.cuda.synchronize()
    K.KernelTimingEnable(False)
    vkern = {}
    for kname in list(abytes) + ["spmv_csr", "ilu_grid_untile", "learned_stage", "ras_apply",
                                 "amg_vcycle"]:
        cnt, ms = K.KernelTimingQuery(kname)
        if cnt == 0 or kname in head_kernels:
            continue
        ent = dict(launches=cnt, total_ms=round(ms, 4), avg_us=round(1000 * ms / cnt, 3))
        if kname in abytes:
            gbs = abytes[kname] / (ms / cnt * 1e-3) / 1e9
            ent.update(bytes_per_launch=abytes[kname], gbs=round(gbs, 1),
                       frac_hbm=round(gbs / HBM_PEAK_GBS, 4))
        vkern[kname] = ent
    for kname, fpc in CONV_FLOPS_PER_CELL.items():
        cnt, ms = K.KernelTimingQuery(kname)
        if cnt:
            tfl = fpc * nb / (ms / cnt * 1e-3) / 1e12
            vkern[kname] = dict(launches=cnt, total_ms=round(ms, 4), avg_us=round(1000 * ms / cnt, 3),
                                flops_per_launch=fpc * nb, tflops=round(tfl, 2),
                                frac_mfma_bf16=round(tfl / MFMA_BF16_PEAK_TFLOPS, 4))

    # dominant kernel of the headline solve (largest total time among the
    # kernels with algorithmic bytes); its average launch over the timed
    # region when the timed region bracketed it, else over the profiling pass
    cand = {k: v for k, v in head_kernels.items() if "bytes_per_launch" in v}
    dom = max(cand, key=lambda k: cand[k]["total_ms"]) if cand else None
    roof = None
    if dom:
        cnt_t, ms_t = timed.get(dom, (0, 0.0))
        if cnt_t:
            avg_us, where, launches = 1000 * ms_t / cnt_t, "timed region", cnt_t
        else:
            avg_us, where, launches = cand[dom]["avg_us"], "profiling pass", cand[dom]["launches"]
        bpl = cand[dom]["bytes_per_launch"]
        ach = round(bpl / (avg_us * 1e-6) / 1e9, 1)
        roof = dict(kernel=dom, bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(ach / HBM_PEAK_GBS, 4),
                    traffic=traffic_from_profiles(dom, args.workload),
                    bytes_per_launch=bpl, avg_launch_us=round(avg_us, 3), launches=launches,
                    measured_in=where)
    # the other candidates as measured in the timed region
    timed_out = {}
    for k, (cnt_t, ms_t) in timed.items():
        if cnt_t and k in abytes:
            us = 1000 * ms_t / cnt_t
            timed_out[k] = dict(sampled_launches=cnt_t, avg_us=round(us, 3),
                                gbs=round(abytes[k] / (us * 1e-6) / 1e9, 1),
                                frac_hbm=round(abytes[k] / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4))

    head = dict(time_s=round(float(np.mean([r["time_s"] for r in results])), 5),
                setup_s=round(float(np.mean([r["setup_s"] for r in results])), 5),
                solve_s=round(float(np.mean([r["solve_s"] for r in results])), 5),
                iters=results[-1]["iters"], true_relres=results[-1]["true_relres"],
                converged=all(r["status"] == 0 for r in results))
    variants = {HEADLINE: head, **variants}

    for S in solvers.values():
        K.SolverDestroy(S)
    K.VecDestroy(bh)
    K.VecDestroy(xh)
    K.MatDestroy(A)
    K.MapDestroy(m)
    for key in ("scalar", "heldout"):
        if key in sys_vecs:
            m1, A1, b1h, x1h = sys_vecs[key][:4]
            K.VecDestroy(b1h)
            K.VecDestroy(x1h)
            K.MatDestroy(A1)
            K.MapDestroy(m1)

    cpu = None
    if not args.no_cpu:
        print("[bench] CPU oracle legs", file=sys.stderr, flush=True)
        cpu = cpu_baseline(s, args.rtol, head["iters"], budget_s=args.cpu_budget)

    ws = 76 * nnzb + 48 * nb + 8 * 31 * n     # matrix + vectors + Krylov basis
    out = {
        "metric": METRIC, "value": head["time_s"], "unit": "s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1000 * t_total / args.steps, 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {wl['desc']}; GMRES(30) + block ILU(0), "
                               f"FP64, rtol {args.rtol:g}, x0 = 0",
                   "headline": HEADLINE, "rtol": args.rtol, "restart": RESTART,
                   "orthogonalization": "lagged CGS2 (two passes over the basis per "
                                        "Arnoldi step; the FGMRES variants keep CGS2)",
                   "step": "assemble + solve of the headline configuration"},
        "iters": head["iters"], "true_relres": head["true_relres"],
        "variants": variants, "kernels": head_kernels, "variant_kernels": vkern,
        "kernels_from": "one untimed headline solve (kernels) and the variants' runs "
                        "(variant_kernels), every instrumented launch bracketed by HIP events",
        "timed_kernels": timed_out,
        "cache": (f"working set {ws / 1e9:.1f} GB, {ws / INFINITY_CACHE_BYTES:.0f}x the 256 MiB "
                  "Infinity Cache: figures are HBM figures" if ws > 4 * INFINITY_CACHE_BYTES
                  else f"working set {ws / 1e6:.0f} MB: kernel figures are cache-resident"
                       + (" (512 MiB flush between steps)" if args.flush else " (not flushed)")),
        "roofline": roof,
        "cpu_baseline": cpu,
        "setup_host": {"generate_s": round(t_gen, 3), "upload_s": round(t_upload, 3)},
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
