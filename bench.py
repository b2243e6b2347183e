"""Benchmark: time to a true FP64 relative residual of 1e-8 on the 64^3
black-oil system, plain FP64 block-ILU(0) against the mixed-precision and
CPR variants, with per-kernel HBM roofline figures and the CPU oracle
timed on the host.

One step = one full pass of the solve path for every configuration in
CONFIGS (preconditioner setup + solve from x0 = 0 each time, inputs
resident in HBM).  The learned-stage configuration loads the trained
network shipped in paper_1701_05913_amd/weights/.  `value` is the mean time-to-solution of the plain
FP64 GMRES(30) + BILU(0) solve; every configuration's time, iterations and
true residual are reported under "variants".

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu]
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

WORKLOADS = {
    "blackoil64": dict(grid=(64, 64, 64), perm="layered", sigma2=2.0,
                       desc="64x64x64 3x3-block black-oil system (786,432 unknowns, "
                            "1,810,432 blocks), layered log-normal permeability, seed 0"),
    "blackoil128x128x64": dict(grid=(128, 128, 64), perm="layered", sigma2=2.0,
                               desc="128x128x64 3x3-block black-oil system "
                                    "(3,145,728 unknowns), seed 0"),
    "channelized256x256x128": dict(grid=(256, 256, 128), perm="channelized", sigma2=3.0,
                                   desc="256x256x128 3x3-block black-oil system (25,165,824 "
                                        "unknowns, 58,458,112 blocks), channelized log-normal "
                                        "permeability (20% channels at 1000x), seed 0"),
    "blackoil32": dict(grid=(32, 32, 32), perm="layered", sigma2=2.0,
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
EXTRAS = {"lgmres30_2_bilu0_f64": dict(aug_k=2), "pcg_ilu0_scalar_f64": dict(system="scalar"),
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
WEIGHTS = os.path.join(ROOT, "paper_1701_05913_amd", "weights", "bilu0_blackoil64.bin")

# matrix-core FLOPs per cell of each conv layer (3x3x3 taps, 2 per MAC)
CONV_FLOPS_PER_CELL = {"conv_l1_fwd": 2 * 27 * 4 * 32, "conv_l2_fwd": 2 * 27 * 32 * 32,
                       "conv_l3_fwd": 2 * 27 * 32 * 32, "conv_l4_fwd": 2 * 27 * 32 * 3}
MFMA_BF16_PEAK_TFLOPS = 2500.0
HEADLINE = "gmres30_bilu0_f64"
# the headline's dominant kernel (the backward block ILU(0) sweep, FP64):
# the only launches the timed region brackets with HIP events
ROOF_KERNEL = "ilu_bwd_bsr3_f64"
ROOF_SAMPLE = 8


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


def traffic_from_profiles(kernel):
    """HBM bytes per launch measured with rocprofv3 FETCH_SIZE/WRITE_SIZE,
    if a summary exists for this kernel and its source has not changed."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        data = json.load(open(path))
        ent = data.get(kernel)
        if not ent:
            return None
        src = os.path.join(ROOT, ent["source"])
        h = hashlib.sha256(open(src, "rb").read()).hexdigest()
        if h != ent["source_sha256"]:
            return None
        return float(ent["bytes_per_launch"])
    except Exception:
        return None


def cpu_baseline(s, rtol, gpu_iters, budget_s=40.0):
    """The FP64 oracle (single-threaded C, as written) on the same system:
    BILU(0) setup + GMRES(30) to rtol.  A 10-iteration prefix sizes the run:
    if the whole solve (about gpu_iters + one restart cycle of iterations)
    fits the budget it runs to the tolerance; otherwise a fixed-iteration
    prefix that fits is timed and scaled to the GPU's iteration count."""
    import oracle
    A = oracle.Matrix.from_system(s)
    t0 = time.perf_counter()
    pc = oracle.PC(A, "bilu0")
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.gmres(A, pc, s["b"], restart=30, maxit=10, rtol=0.0, fixed_iters=True)
    per_it = (time.perf_counter() - t0) / 10
    if t_setup + per_it * (gpu_iters + 30) < budget_s:
        t0 = time.perf_counter()
        r = oracle.gmres(A, pc, s["b"], restart=30, maxit=5000, rtol=rtol)
        t_solve = time.perf_counter() - t0
        return dict(value=round(t_setup + t_solve, 4), unit="s", cores=1, kind="oracle",
                    iters=r["iters"], true_relres=r["relres"],
                    sample="the whole workload: BILU(0) setup + GMRES(30) solve to the same "
                           "rtol, single-threaded oracle")
    k = max(10, int((budget_s - t_setup) / per_it))
    t0 = time.perf_counter()
    oracle.gmres(A, pc, s["b"], restart=30, maxit=k, rtol=0.0, fixed_iters=True)
    per_it = (time.perf_counter() - t0) / k
    return dict(value=round(t_setup + per_it * gpu_iters, 4), unit="s", cores=1, kind="oracle",
                sample=f"BILU(0) setup + {k} GMRES(30) iterations timed, scaled to the GPU's "
                       f"{gpu_iters} iterations, single-threaded oracle")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="blackoil64", choices=sorted(WORKLOADS))
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--configs", default="all")
    ap.add_argument("--layout", default="auto", choices=["auto", "levels", "grid"],
                    help="ILU sweep layout (see SolverSetSweepLayout)")
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
    t0 = time.perf_counter()
    s = ri.blackoil_system(*wl["grid"], seed=0, perm=wl["perm"], sigma2=wl["sigma2"])
    t_gen = time.perf_counter() - t0
    nb = len(s["rowptr"]) - 1
    n = 3 * nb
    nnzb = int(s["rowptr"][-1])
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(np.ascontiguousarray(s["rowptr"], dtype=np.int32)).to(dev)
    ci = torch.from_numpy(np.ascontiguousarray(s["col"], dtype=np.int32)).to(dev)
    va = torch.from_numpy(np.ascontiguousarray(s["val"].reshape(-1))).to(dev)
    b = torch.from_numpy(s["b"]).to(dev)
    x = torch.zeros(n, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    K.KrylovSetStream(stream)
    m = K.MapCreateLocal(n)
    t0 = time.perf_counter()
    A = K.MatCreateBSR(m, nb, 3, rp, ci, va)
    torch.cuda.synchronize()
    t_upload = time.perf_counter() - t0
    bh, xh = K.VecWrap(m, b), K.VecWrap(m, x)
    lnk = torch.from_numpy(np.asarray(s["lnk"], dtype=np.float32)).to(dev)

    configs = CONFIGS if args.configs == "all" else [c for c in CONFIGS if c[0] in args.configs.split(",")]
    # the scalar system, built only when a configuration needs it
    sys_vecs = {"blackoil": (m, A, bh, xh, x)}
    if any(EXTRAS.get(c[0], {}).get("system") == "scalar" for c in configs):
        ss = ri.scalar_system(*wl["grid"], seed=0)
        ns = len(ss["rowptr"]) - 1
        m1 = K.MapCreateLocal(ns)
        A1 = K.MatCreateCSR(m1, ns, torch.from_numpy(np.ascontiguousarray(ss["rowptr"], dtype=np.int32)).to(dev),
                            torch.from_numpy(np.ascontiguousarray(ss["col"], dtype=np.int32)).to(dev),
                            torch.from_numpy(np.ascontiguousarray(ss["val"].reshape(-1))).to(dev))
        b1 = torch.from_numpy(ss["b"]).to(dev)
        x1 = torch.zeros(ns, dtype=torch.float64, device=dev)
        sys_vecs["scalar"] = (m1, A1, K.VecWrap(m1, b1), K.VecWrap(m1, x1), x1)
    solvers = {}
    for name, st, pc, prec, cpr in configs:
        ex = EXTRAS.get(name, {})
        mm, AA = sys_vecs[ex.get("system", "blackoil")][:2]
        S = K.SolverCreate(getattr(K, f"KRY_{st}"), getattr(K, f"KRY_PC_{pc}"), mm)
        K.SolverSetMat(S, AA)
        K.SolverSetRtol(S, args.rtol)
        K.SolverSetMaxit(S, 5000)
        K.SolverSetRestart(S, 30)
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
        K.SolverSetSweepLayout(S, getattr(K, f"KRY_SWEEP_{args.layout.upper()}"))
        if pc.endswith("_LEARNED"):
            K.SolverSetLearned(S, WEIGHTS, lnk)
        solvers[name] = S

    def run_one(name):
        S = solvers[name]
        _, _, bv, xv, xt = sys_vecs[EXTRAS.get(name, {}).get("system", "blackoil")]
        xt.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        K.SolverAssemble(S)
        rc = K.SolverSolve(S, bv, xv)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st, ss = K.SolverGetTimes(S)
        out = dict(time_s=dt, setup_s=st, solve_s=ss, iters=K.SolverGetIters(S),
                   true_relres=K.SolverGetResidual(S), status=rc)
        if name.endswith("_learned"):
            out["stage_applies"], out["stage_fallbacks"] = K.SolverGetLearnedStats(S)
        print(f"[bench] {name}: {dt:.4f} s, {out['iters']} iterations", file=sys.stderr, flush=True)
        return out

    for _ in range(args.warmup):
        for name, *_ in configs:
            run_one(name)

    # timed region: HIP events bracket only the headline's dominant kernel,
    # one launch in every ROOF_SAMPLE (every event adds a few microseconds
    # between the launches it separates)
    K.KernelTimingReset()
    K.KernelTimingSelect(ROOF_KERNEL)
    K.KernelTimingSample(ROOF_SAMPLE)
    K.KernelTimingEnable(True)
    results = {name: [] for name, *_ in configs}
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        for name, *_ in configs:
            results[name].append(run_one(name))
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    K.KernelTimingEnable(False)
    roof_cnt, roof_ms = K.KernelTimingQuery(ROOF_KERNEL)

    # per-kernel figures: one more, untimed pass of every configuration with
    # every instrumented launch bracketed
    K.KernelTimingReset()
    K.KernelTimingSelect(None)
    K.KernelTimingSample(1)
    K.KernelTimingEnable(True)
    for name, *_ in configs:
        run_one(name)
    torch.cuda.synchronize()
    K.KernelTimingEnable(False)
    abytes = algorithmic_bytes(nb, nnzb)
    kernels = {}
    for kname in list(abytes) + ["cgs2", "ilu_fwd_csr_f64", "ilu_bwd_csr_f64",
                                 "ilu_fwd_csr_f32", "ilu_bwd_csr_f32", "spmv_csr"]:
        cnt, ms = K.KernelTimingQuery(kname)
        if cnt == 0:
            continue
        ent = dict(launches=cnt, total_ms=round(ms, 4), avg_us=round(1000 * ms / cnt, 3))
        if kname in abytes:
            gbs = abytes[kname] / (ms / cnt * 1e-3) / 1e9
            ent.update(bytes_per_launch=abytes[kname], gbs=round(gbs, 1),
                       frac_hbm=round(gbs / HBM_PEAK_GBS, 4))
        kernels[kname] = ent
    for kname in ["ilu_grid_untile", "learned_stage", "ras_apply", "ras_ilu_fwd", "ras_ilu_bwd",
                  "amg_vcycle"]:
        cnt, ms = K.KernelTimingQuery(kname)
        if cnt:
            kernels[kname] = dict(launches=cnt, total_ms=round(ms, 4), avg_us=round(1000 * ms / cnt, 3))
    for kname, fpc in CONV_FLOPS_PER_CELL.items():
        cnt, ms = K.KernelTimingQuery(kname)
        if cnt:
            tfl = fpc * nb / (ms / cnt * 1e-3) / 1e12
            kernels[kname] = dict(launches=cnt, total_ms=round(ms, 4), avg_us=round(1000 * ms / cnt, 3),
                                  flops_per_launch=fpc * nb, tflops=round(tfl, 2),
                                  frac_mfma_bf16=round(tfl / MFMA_BF16_PEAK_TFLOPS, 4))
    # dominant kernel of the headline configuration's families
    cand = {k: v for k, v in kernels.items() if k in abytes}
    dom = max(cand, key=lambda k: cand[k]["total_ms"]) if cand else None
    roof = None
    if dom:
        # the dominant kernel's average launch over the timed region when
        # that is the kernel the timed region bracketed, else over the
        # profiling pass
        if dom == ROOF_KERNEL and roof_cnt:
            avg_us, where = 1000 * roof_ms / roof_cnt, "timed region"
        else:
            avg_us, where = cand[dom]["avg_us"], "profiling pass"
        ach = round(abytes[dom] / (avg_us * 1e-6) / 1e9, 1)
        roof = dict(kernel=dom, bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(ach / HBM_PEAK_GBS, 4), traffic=traffic_from_profiles(dom),
                    bytes_per_launch=abytes[dom], avg_launch_us=round(avg_us, 3),
                    launches=roof_cnt if where == "timed region" else cand[dom]["launches"],
                    measured_in=where)

    variants = {}
    for name, *_ in configs:
        rs = results[name]
        variants[name] = dict(
            time_s=round(float(np.mean([r["time_s"] for r in rs])), 5),
            setup_s=round(float(np.mean([r["setup_s"] for r in rs])), 5),
            solve_s=round(float(np.mean([r["solve_s"] for r in rs])), 5),
            iters=rs[-1]["iters"], true_relres=rs[-1]["true_relres"],
            converged=all(r["status"] == 0 for r in rs))
        if "stage_applies" in rs[-1]:
            variants[name].update(stage_applies=rs[-1]["stage_applies"],
                                  stage_fallbacks=rs[-1]["stage_fallbacks"])
    head = variants.get(HEADLINE) or next(iter(variants.values()))

    for S in solvers.values():
        K.SolverDestroy(S)
    K.VecDestroy(bh)
    K.VecDestroy(xh)
    K.MatDestroy(A)
    K.MapDestroy(m)
    if "scalar" in sys_vecs:
        m1, A1, b1h, x1h, _ = sys_vecs["scalar"]
        K.VecDestroy(b1h)
        K.VecDestroy(x1h)
        K.MatDestroy(A1)
        K.MapDestroy(m1)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(s, args.rtol, head["iters"])

    out = {
        "metric": METRIC, "value": head["time_s"], "unit": "s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1000 * t_total / args.steps, 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {wl['desc']}; GMRES(30) + block ILU(0), "
                               f"FP64, rtol {args.rtol:g}, x0 = 0",
                   "headline": HEADLINE, "rtol": args.rtol, "restart": 30,
                   "sweep_layout": args.layout,
                   "step": "assemble + solve of every configuration in variants"},
        "iters": head["iters"], "true_relres": head["true_relres"],
        "variants": variants, "kernels": kernels,
        "kernels_from": "one untimed pass of every configuration, every instrumented launch "
                        "bracketed by HIP events",
        "roofline": roof,
        "cpu_baseline": cpu,
        "setup_host": {"generate_s": round(t_gen, 3), "upload_s": round(t_upload, 3)},
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
