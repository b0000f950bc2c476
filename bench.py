"""Benchmark: RSAI(tol) construction throughput on one MI355X.

Workload: the 2D 5-point upwind convection-diffusion matrix on a 512 x 512 grid
(n = 262144, nnz = 1,308,672), per-cell convection uniform in [-50, 50]^2 * h from
seed 0; RSAI parameters c = 3, lmax = 8, eps = 0.4, fixed drop tolerance 1e-3.
A step is one complete rsai_build (CSC check, row pattern, the fused size-tiered
RSAI kernels, assembly of M as CSC) on inputs already resident in HBM.

Printed as one JSON line: columns/s of the batched schedule (the value), the
plain schedule on the same GPU, fwd+bwd time of the loss
sum_k ||A m_k - e_k||^2 + ||A M b - b||^2, the roofline of the dominant kernel
(HIP events around it on its own stream), and the CPU oracle on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "RSAI columns/sec (FP64, n=262k) batched vs plain; fwd+bwd time; % FP64 roofline"
FP64_PEAK_TFLOPS = 78.6   # MI355X FP64 vector: 256 CU x 2.4 GHz x 128 flop/clk
HBM_PEAK_GBS = 8000.0
PARAMS = dict(c=3, lmax=8, eps=0.4, drop="fixed", tol=1e-3, validate=2)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--grid", type=int, default=512)
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the power-law (n = 10^6), 64-matrix batch and 3D fwd+bwd legs")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 64 MiB device to device three times (calibrates the HBM byte counters)")
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="only run this many batched builds (for rocprofv3), print nothing else")
    ap.add_argument("--profile-workload", choices=("cd2d", "batch64", "bicgstab", "fwdbwd", "eps02", "powerlaw"),
                    default="cd2d",
                    help="workload of --profile-steps: builds of the cd2d matrix (eps 0.4, or eps02: 0.2), "
                         "of the power-law matrix (n = 10^6) or of the 64-matrix batch, BiCGStab solves "
                         "(100 iterations) with M of the cd2d matrix, or fwd + bwd steps of the loss on the "
                         "cd2d matrix")
    return ap.parse_args()


def measured_traffic():
    """HBM bytes per launch of the tier-0 kernel from the committed rocprofv3 counter
    summary, if it was taken on the current kernel sources (else None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "tier_kernel_cd2d512_pmc.md")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and line.startswith("    ") and not line.strip().startswith("rocprofv3"):
            k, v = line.strip().split(":", 1)
            kv[k.strip()] = v.strip()
    h = hashlib.sha256()
    for f in ("rsai_tier.hip", "rsai_tier_kernel.h", "rsai_tier.h", "rsai_dev.h"):
        with open(os.path.join(ROOT, "paper_1503_04500_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if kv.get("kernel_source_sha256") != h.hexdigest() or "traffic_bytes_per_launch" not in kv:
        return None
    return float(kv["traffic_bytes_per_launch"])


def alg_bytes(n, nnz, nnzM):
    """Compulsory HBM bytes of a build's size-class kernels: A (values, row indices,
    column pointers) and its row pattern (column indices, row pointers) read once, the
    results (row indices and values of M) and the per-column statistics written once."""
    return (nnz * (8 + 4) + (n + 1) * 8) + (nnz * 4 + (n + 1) * 8) + nnzM * (4 + 8) + n * (8 + 4 * 4 + 8 * 3)


def class_roofline(rsai, mats, prm, np):
    """Roofline of the size-class kernels of one (batched) build: model flops of every
    column and compulsory bytes over the HIP-event time of those kernels."""
    p = rsai.build_batched(mats, timing=True, **prm)
    nz = [p.nnz(i) for i in range(len(mats))]
    t = p.timing()
    fl = sum(float(p.stats(i, fields=("flops",))["flops"].sum().item()) for i in range(len(mats)))
    by = sum(alg_bytes(m.n, m.nnz, z) for m, z in zip(mats, nz))
    p.close()
    ms = t["tier0"] + t["tiers"]
    tf = fl / (ms * 1e-3) / 1e12
    gbs = by / (ms * 1e-3) / 1e9
    return {"bound": "alu", "achieved": tf, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": tf / FP64_PEAK_TFLOPS, "kernel": "the size-class kernels (tier 0, later tiers, sparse-block "
                                                       "and dense classes)", "kernel_ms": ms, "alg_flops": fl,
            "hbm_alg_bytes": by, "hbm_achieved_GBs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS, "traffic": None,
            "note": "the flops are the dense Householder-update model; the sparse-block class solves an "
                    "orthogonally compressed block with fewer operations, so its share is an upper bound"}


def adjoint_roofline(rsai, A, H, torch, np, prm):
    """Roofline of the adjoint kernels on kept factors: z = R^-1 R^-T g (two triangular
    solves, 2 q^2), r and A_k z over the entries of the columns of J (4 each) and the
    contribution per entry (6); compulsory bytes: the R records, M, g and A read once,
    dA read and written once."""
    p = rsai.build(A, timing=True, keep_factors=True, **prm)
    cp, ri, va = p.export()
    cpn, rin = cp.cpu().numpy(), ri.cpu().numpy()
    g = torch.cos(torch.arange(va.numel(), dtype=torch.float64, device=va.device))
    dA = torch.zeros(H.nnz, dtype=torch.float64, device=va.device)
    ms = []
    for _ in range(4):
        p.backward(g, 1.0, dA)
        ms.append(p.timing()["backward"])
    p.close()
    q = np.diff(cpn).astype(np.float64)
    lens = np.diff(H.colptr).astype(np.float64)
    ent = lens[rin]                                  # entries of column j of A, per entry of M
    fl = float(np.sum(2.0 * q * q) + 10.0 * ent.sum())
    by = float(8 * np.sum(q + q * (q + 1) / 2) + 12 * cpn[-1] + 8 * cpn[-1] + 12 * H.nnz + 8 * (H.n + 1)
               + 16 * H.nnz)
    t = float(np.median(ms[1:]))
    tf = fl / (t * 1e-3) / 1e12
    gbs = by / (t * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
            "kernel": "backward_factored_kernel<16,32,1>", "kernel_ms": t, "hbm_alg_bytes": by,
            "alg_flops": fl, "fp64_TFLOPs": tf, "fp64_frac": tf / FP64_PEAK_TFLOPS, "traffic": None}


def time_builds(rsai, A, sched, steps, warmup, torch, prm=None):
    prm = PARAMS if prm is None else prm
    for _ in range(warmup):
        p = rsai.build(A, sched=sched, **prm)
        p.nnz()
        p.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = None
    for _ in range(steps):
        if plan is not None:
            plan.close()
        plan = rsai.build(A, sched=sched, **prm)
        plan.nnz()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    plan.close()
    return dt


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(columns are independent; the sharding design is described in DESIGN.md).", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    if args.copy_probe:
        a = torch.ones(64 * 1024 * 1024 // 8, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": a.numel() * 8, "copies": 3}))
        return

    import paper_1503_04500_amd.rsai as rsai
    from paper_1503_04500_amd import gen

    if args.profile_steps and args.profile_workload == "batch64":
        A5 = [rsai.Matrix.from_host(gen.make(sp), "cuda:0") for sp in gen.batch64_specs()]
        for _ in range(args.profile_steps):
            p = rsai.build_batched(A5, **PARAMS)
            p.nnz()
            p.close()
        torch.cuda.synchronize()
        print(json.dumps({"profile_steps": args.profile_steps, "workload": "batch64"}))
        return

    if args.profile_steps and args.profile_workload == "powerlaw":
        A3 = rsai.Matrix.from_host(gen.c3(), "cuda:0")
        for _ in range(args.profile_steps):
            p = rsai.build(A3, **dict(PARAMS, lmax=10))
            p.nnz()
            p.close()
        torch.cuda.synchronize()
        print(json.dumps({"profile_steps": args.profile_steps, "workload": "powerlaw"}))
        return

    H = gen.cd2d(args.grid, seed=0)
    A = rsai.Matrix.from_host(H, "cuda:0")
    torch.cuda.synchronize()

    if args.profile_steps and args.profile_workload == "eps02":
        for _ in range(args.profile_steps):
            p = rsai.build(A, **dict(PARAMS, eps=0.2))
            p.nnz()
            p.close()
        torch.cuda.synchronize()
        print(json.dumps({"profile_steps": args.profile_steps, "workload": "eps02"}))
        return

    if args.profile_steps and args.profile_workload == "bicgstab":
        pb = rsai.build(A, sched="batched", **PARAMS)
        pb.nnz()
        bvec = rsai.spmv(A, torch.ones(H.n, dtype=torch.float64, device="cuda:0"))
        for _ in range(args.profile_steps):
            _, its, _ = pb.bicgstab(bvec, maxit=100)
        torch.cuda.synchronize()
        pb.close()
        print(json.dumps({"profile_steps": args.profile_steps, "workload": "bicgstab", "iterations": its}))
        return

    if args.profile_steps and args.profile_workload == "fwdbwd":
        from paper_1503_04500_amd import autograd as ag
        bv = torch.from_numpy(np.random.default_rng(0).standard_normal(H.n)).to("cuda:0")
        for _ in range(args.profile_steps):
            val = A.val.clone().requires_grad_(True)
            ag.rsai_loss(A, val, bv, **PARAMS).backward()
        torch.cuda.synchronize()
        print(json.dumps({"profile_steps": args.profile_steps, "workload": "fwdbwd"}))
        return

    if args.profile_steps:
        for _ in range(args.profile_steps):
            p = rsai.build(A, sched="batched", **PARAMS)
            p.nnz()
            p.close()
        torch.cuda.synchronize()
        print(json.dumps({"profile_steps": args.profile_steps}))
        return

    # ---- batched (the value)
    dt_b = time_builds(rsai, A, "batched", args.steps, args.warmup, torch)
    # ---- dominant kernel timing with HIP events on the build stream, plus stats
    tier0_ms, kern_ms, build_ms = [], [], []
    last = None
    for _ in range(max(3, min(args.steps, 10))):
        if last is not None:
            last.close()
        last = rsai.build(A, sched="batched", timing=True, **PARAMS)
        t = last.timing()
        tier0_ms.append(t["tier0"])
        kern_ms.append(t["tier0"] + t["tiers"])
        build_ms.append(t["build"])
    st = {k: v.cpu().numpy() for k, v in last.stats().items()}
    nnzM = last.nnz()
    last.close()
    flops = float(st["flops"].sum())
    t0_ms = float(np.median(tier0_ms))
    k_ms = float(np.median(kern_ms))
    # the model flops of every column over the time of every size-class kernel of the
    # build (tier 0 and the later classes, which finish the columns that leave it)
    achieved_tf = flops / (k_ms * 1e-3) / 1e12
    n, nnz = H.n, H.nnz
    bytes_alg = alg_bytes(n, nnz, nnzM)
    hbm_gbs = bytes_alg / (k_ms * 1e-3) / 1e9

    # ---- the same build replayed as a captured HIP graph on the plan's buffers
    # (rsai_rebuild: no allocation, no host-side setup)
    gp = rsai.build(A, sched="batched", **PARAMS)
    gp.nnz()
    for _ in range(args.warmup + 1):
        gp.rebuild(graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        gp.rebuild(graph=True)
    torch.cuda.synchronize()
    dt_g = (time.perf_counter() - t0) / args.steps
    graph = {"value": H.n / dt_g, "ms_per_step": dt_g * 1e3, "unit": "columns/s",
             "nnzM_equal": gp.nnz() == nnzM}
    gp.close()

    # ---- plain schedule
    plain = None
    if not args.no_plain:
        dt_p = time_builds(rsai, A, "plain", max(3, args.steps // 4), 1, torch)
        plain = {"value": n / dt_p, "ms_per_step": dt_p * 1e3, "unit": "columns/s"}

    # ---- fwd + bwd of L = sum_k ||A m_k - e_k||^2 + ||A M b - b||^2
    from paper_1503_04500_amd import autograd as ag
    b = torch.from_numpy(np.random.default_rng(0).standard_normal(n)).to("cuda:0")
    fb = []
    for it in range(4):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        val = A.val.clone().requires_grad_(True)
        L = ag.rsai_loss(A, val, b, **PARAMS)
        L.backward()
        torch.cuda.synchronize()
        if it > 0:
            fb.append(time.perf_counter() - t0)
    fwd_bwd_ms = float(np.median(fb)) * 1e3
    adj_roof = adjoint_roofline(rsai, A, H, torch, np, PARAMS)

    # ---- further workloads (reported beside the value): power-law n = 10^6, the
    # 64-matrix batch in one build, fwd+bwd on the 64^3 3D matrix
    extra = None
    host_mats = {}  # host copies of the other workloads, for the CPU oracle's legs
    if not args.no_extra:
        extra = {}
        # right-preconditioned BiCGStab on the device with this M (x0 = 0, b = A*1,
        # stop at ||b - A x|| / ||b|| < 1e-8), and without a preconditioner
        pb = rsai.build(A, sched="batched", **PARAMS)
        pb.nnz()
        bvec = rsai.spmv(A, torch.ones(n, dtype=torch.float64, device="cuda:0"))
        sol = {}
        for key, pre in (("rsai", True), ("none", False)):
            pb.bicgstab(bvec, precond=pre)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(3):
                _, its, rel = pb.bicgstab(bvec, precond=pre)
            dts = (time.perf_counter() - t0) / 3
            sol[key] = {"iterations": its, "relres": rel, "ms": dts * 1e3,
                        "us_per_iteration": dts * 1e6 / max(its, 1)}
        pb.close()
        # the left form: RSAI on A^T (its build timed too), M A x = M b
        At = A.transpose()
        dtt = time_builds(rsai, At, "batched", 3, 1, torch)
        pt = rsai.build(At, sched="batched", **PARAMS)
        pt.nnz()
        rsai.bicgstab_left(A, pt, bvec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            _, its, rel = rsai.bicgstab_left(A, pt, bvec)
        dts = (time.perf_counter() - t0) / 3
        sol["rsai_left"] = {"iterations": its, "relres": rel, "ms": dts * 1e3,
                            "us_per_iteration": dts * 1e6 / max(its, 1), "build_on_At_ms": dtt * 1e3}
        pt.close()
        del At
        extra["bicgstab_cd2d512"] = sol
        # the stopping criterion, the number of dominant indices and the dropping mode
        # varied on the same matrix: density of M, columns left above eps, build time,
        # device BiCGStab iterations and time
        sweep = []
        for eps, c, drop in ((0.5, 3, "fixed"), (0.4, 3, "fixed"), (0.3, 3, "fixed"), (0.2, 3, "fixed"),
                             (0.4, 1, "fixed"), (0.4, 5, "fixed"), (0.4, 3, "adaptive"), (0.4, 3, "none")):
            prm = dict(PARAMS, eps=eps, c=c, drop=drop)
            dt = time_builds(rsai, A, "batched", 3, 1, torch, prm=prm)
            ps = rsai.build(A, sched="batched", **prm)
            nzm = ps.nnz()
            rn = ps.stats()["resnorm"]
            t0 = time.perf_counter()
            _, its, rel = ps.bicgstab(bvec)
            dts = time.perf_counter() - t0
            sweep.append({"eps": eps, "c": c, "drop": drop, "build_ms": dt * 1e3, "spar": nzm / nnz,
                          "n_c": int((rn > eps).sum().item()), "bicgstab_iterations": its,
                          "bicgstab_ms": dts * 1e3})
            ps.close()
        extra["sweep_cd2d512"] = sweep
        # eps = 0.1 (the paper's smallest setting): blocks of about 100 x 64, most columns
        # end in the workgroup classes; on the 128x128 grid
        H01 = gen.cd2d(128, seed=0)
        A01 = rsai.Matrix.from_host(H01, "cuda:0")
        prm01 = dict(PARAMS, eps=0.1)
        dt01 = time_builds(rsai, A01, "batched", 3, 1, torch, prm=prm01)
        p01 = rsai.build(A01, sched="batched", timing=True, **prm01)
        nz01 = p01.nnz()
        b01 = rsai.spmv(A01, torch.ones(H01.n, dtype=torch.float64, device="cuda:0"))
        _, its01, _ = p01.bicgstab(b01)
        extra["eps01_cd2d128"] = {"eps": 0.1, "c": 3, "build_ms": dt01 * 1e3, "spar": nz01 / H01.nnz,
                                  "phase_ms": p01.timing(), "bicgstab_iterations": its01,
                                  "workload": "cd2d 128x128 seed 0; c=3 lmax=8 eps=0.1 tol=1e-3"}
        p01.close()
        del A01, H01
        # eps = 0.1 on the benchmark's 512x512 grid: about 243000 columns pass the
        # sparse-block class to the dense class, whose queues must then hold every column
        # (spill_capacity = n); one timed build
        prm01b = dict(PARAMS, eps=0.1, spill_capacity=H.n)
        dt01b = time_builds(rsai, A, "batched", 1, 1, torch, prm=prm01b)
        p01b = rsai.build(A, sched="batched", **prm01b)
        nz01b = p01b.nnz()
        _, its01b, _ = p01b.bicgstab(rsai.spmv(A, torch.ones(H.n, dtype=torch.float64, device="cuda:0")))
        extra["eps01_cd2d512"] = {"eps": 0.1, "c": 3, "build_ms": dt01b * 1e3, "spar": nz01b / H.nnz,
                                  "bicgstab_iterations": its01b, "spill_capacity": H.n,
                                  "workload": "cd2d 512x512 seed 0; c=3 lmax=8 eps=0.1 tol=1e-3"}
        p01b.close()
        # relatively dense rows (Section 4): 512x512 grid plus 1024 rows of 32 entries
        Hd = gen.dense_rows(512, 1024, 32)
        Ad = rsai.Matrix.from_host(Hd, "cuda:0")
        dtd = time_builds(rsai, Ad, "batched", 5, 1, torch)
        pdn = rsai.build(Ad, sched="batched", timing=True, **PARAMS)
        pdn.nnz()
        extra["dense_rows_512"] = {"value": Hd.n / dtd, "unit": "columns/s", "ms_per_step": dtd * 1e3,
                                   "phase_ms": pdn.timing(),
                                   "workload": "cd2d 512x512 seed 0 plus 1024 rows of 32 entries U(-1,1), "
                                               "seed 7919; RSAI(tol) c=3 lmax=8 eps=0.4 tol=1e-3"}
        pdn.close()
        del Ad, Hd
        P3 = dict(PARAMS, lmax=10)
        H3 = gen.c3()
        A3 = rsai.Matrix.from_host(H3, "cuda:0")
        dt3 = time_builds(rsai, A3, "batched", 3, 1, torch, prm=P3)
        extra["powerlaw_1e6"] = {"value": H3.n / dt3, "unit": "columns/s", "ms_per_step": dt3 * 1e3,
                                 "workload": "power-law columns (min 2, mean 7, max 200), n=10^6, seed 0; "
                                             "c=3 lmax=10 eps=0.4 tol=1e-3",
                                 "roofline": class_roofline(rsai, [A3], P3, np)}
        # the plain schedule (one launch per loop; its outgrown columns go on to the same
        # workgroup classes) on the deeper workloads, beside the batched one
        dt3p = time_builds(rsai, A3, "plain", 2, 1, torch, prm=P3)
        dt02p = time_builds(rsai, A, "plain", 2, 1, torch, prm=dict(PARAMS, eps=0.2))
        dt02b = time_builds(rsai, A, "batched", 2, 1, torch, prm=dict(PARAMS, eps=0.2))
        extra["plain_vs_batched"] = {
            "powerlaw_1e6": {"plain_ms": dt3p * 1e3, "batched_ms": dt3 * 1e3, "speedup": dt3p / dt3},
            "cd2d512_eps0.2": {"plain_ms": dt02p * 1e3, "batched_ms": dt02b * 1e3, "speedup": dt02p / dt02b}}
        host_mats["c3"] = H3
        del A3, H3
        specs = gen.batch64_specs()
        H5 = [gen.make(sp) for sp in specs]
        A5 = [rsai.Matrix.from_host(h, "cuda:0") for h in H5]
        n5 = sum(h.n for h in H5)
        for _ in range(1):
            p5 = rsai.build_batched(A5, **PARAMS)
            p5.nnz()
            p5.close()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            p5 = rsai.build_batched(A5, **PARAMS)
            p5.nnz()
            p5.close()
        torch.cuda.synchronize()
        dt5 = (time.perf_counter() - t0) / 3
        # the same 64 matrices built one after another, and the batched build replayed
        # as a captured graph
        torch.cuda.synchronize()
        per5 = []
        t0 = time.perf_counter()
        for a5 in A5:
            t1 = time.perf_counter()
            p1 = rsai.build(a5, **PARAMS)
            p1.nnz()
            p1.close()
            per5.append((time.perf_counter() - t1) * 1e3)
        torch.cuda.synchronize()
        dt5s = time.perf_counter() - t0
        p5 = rsai.build_batched(A5, **PARAMS)
        p5.nnz()
        p5.rebuild(graph=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            p5.rebuild(graph=True)
        torch.cuda.synchronize()
        dt5g = (time.perf_counter() - t0) / 3
        p5.close()
        extra["batch64"] = {"value": n5 / dt5, "unit": "columns/s", "ms_per_step": dt5 * 1e3,
                            "roofline": class_roofline(rsai, A5, PARAMS, np),
                            "sequential_ms": dt5s * 1e3, "graph_replay_ms": dt5g * 1e3,
                            "sequential_per_matrix_ms": [round(v, 3) for v in per5],
                            "workload": f"64 matrices in one build (2D/3D convection-diffusion, power-law; "
                                        f"sum n = {n5})"}
        # fwd + bwd of the summed loss over the 64 matrices (one batched build keeping
        # R factors in the default 256 MB store, one adjoint per matrix; the columns
        # past the store get their factor recomputed)
        b5 = [torch.from_numpy(np.random.default_rng(2000 + i).standard_normal(h.n)).to("cuda:0")
              for i, h in enumerate(H5)]
        fb5 = []
        for it in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            v5 = [a5.val.clone().requires_grad_(True) for a5 in A5]
            L5 = ag.rsai_loss_batched(A5, v5, b5, **PARAMS)
            L5.backward()
            torch.cuda.synchronize()
            if it > 0:
                fb5.append(time.perf_counter() - t0)
            del v5, L5
        extra["batch64"]["fwd_bwd_ms"] = float(np.median(fb5)) * 1e3
        host_mats["c5"] = H5
        del A5, H5
        H4 = gen.c4()
        A4 = rsai.Matrix.from_host(H4, "cuda:0")
        b4 = torch.from_numpy(np.random.default_rng(0).standard_normal(H4.n)).to("cuda:0")
        fb4 = []
        for it in range(4):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            val = A4.val.clone().requires_grad_(True)
            L = ag.rsai_loss(A4, val, b4, **PARAMS)
            L.backward()
            torch.cuda.synchronize()
            if it > 0:
                fb4.append(time.perf_counter() - t0)
        extra["fwd_bwd_cd3d64_ms"] = float(np.median(fb4)) * 1e3
        host_mats["c4"] = H4
        del A4, H4

    # ---- CPU oracle on the host cores (full matrix, repeated up to ~10 s)
    cpu = None
    if not args.no_cpu:
        import oracle
        reps, tot, thr = 0, 0.0, 0
        while tot < 10.0 and reps < 200:
            R = oracle.rsai(H, c=3, lmax=8, eps=0.4, drop=oracle.DROP_FIXED, tol=1e-3)
            tot += R["seconds"]
            thr = R["threads"]
            reps += 1
        cpu = {"value": reps * n / tot, "unit": "columns/s", "cores": int(thr), "kind": "oracle",
               "sample": f"the full {args.grid}x{args.grid} matrix ({n} columns) built {reps} times"}
        # end to end (Section 5 protocol, b = A 1): the host BiCGStab with the oracle's M
        # and with the GPU's M, beside the device solve with the GPU's M
        pe = rsai.build(A, sched="batched", **PARAMS)
        gM = tuple(t.cpu().numpy() for t in pe.export())
        bh = H.matvec(np.ones(n))
        _, it_dev, _ = pe.bicgstab(torch.from_numpy(bh).to("cuda:0"))
        pe.close()
        it_om, rel_om, _ = oracle.bicgstab(H, bh, (R["colptr"], R["rowidx"], R["val"]))
        it_gm, rel_gm, _ = oracle.bicgstab(H, bh, gM)
        cpu["e2e_bicgstab"] = {"oracle_M_host_solver": it_om, "gpu_M_host_solver": it_gm,
                               "gpu_M_device_solver": it_dev, "same_pattern": bool(np.array_equal(gM[1], R["rowidx"]))}
        # one host thread, on a seeded sample of 32768 columns
        cols = np.sort(np.random.default_rng(0).choice(n, 32768, replace=False))
        R1 = oracle.rsai(H, c=3, lmax=8, eps=0.4, drop=oracle.DROP_FIXED, tol=1e-3, threads=1, cols=cols)
        cpu["one_core"] = {"value": cols.size / R1["seconds"], "unit": "columns/s", "cores": 1,
                           "sample": "32768 seeded columns of the same matrix"}
        # the other workloads: the 32x32 and 64^3 matrices in full, the power-law
        # matrix and the 64-matrix batch on seeded column samples (seconds each)
        # (the thread count is passed explicitly: the one-thread run above leaves it at 1)
        P_o = dict(c=3, lmax=8, eps=0.4, drop=oracle.DROP_FIXED, tol=1e-3, threads=int(thr))

        def oracle_leg(mats, kw, per):
            secs, k, thr = 0.0, 0, 0
            for i, Hx in enumerate(mats):
                cs = None
                if per is not None and per < Hx.n:
                    cs = np.sort(np.random.default_rng(i).choice(Hx.n, per, replace=False))
                Rx = oracle.rsai(Hx, cols=cs, **kw)
                secs += Rx["seconds"]
                k += Hx.n if cs is None else cs.size
                thr = Rx["threads"]
            return {"value": k / secs, "unit": "columns/s", "cores": int(thr), "columns": int(k),
                    "of": int(sum(Hx.n for Hx in mats))}

        by = {"cd2d_32x32": oracle_leg([gen.c1()], P_o, None)}
        if "c4" in host_mats:
            by["cd3d_64"] = oracle_leg([host_mats["c4"]], P_o, None)
        if "c3" in host_mats:
            by["powerlaw_1e6"] = dict(oracle_leg([host_mats["c3"]], dict(P_o, lmax=10), 20000),
                                      sample="20000 seeded columns")
        if "c5" in host_mats:
            by["batch64"] = dict(oracle_leg(host_mats["c5"], P_o, 1000),
                                 sample="1000 seeded columns of each of the 64 matrices")
        cpu["by_workload"] = by

    # peaks measured on this device, beside the published ones: the FP64 FMA loop of
    # the library and a device-to-device copy of 1 GiB (read + write counted)
    fma_tf = rsai.peak_fp64()
    ca = torch.empty(1 << 27, dtype=torch.float64, device="cuda:0")
    cb = torch.empty_like(ca)
    cb.copy_(ca)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        cb.copy_(ca)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 10 * 2 * ca.numel() * 8 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del ca, cb
    measured = {"fp64_fma_TFLOPs": fma_tf, "hbm_copy_GBs": copy_gbs,
                "frac_of_measured_fp64": achieved_tf / fma_tf, "hbm_frac_of_measured_copy": hbm_gbs / copy_gbs}

    out = {
        "metric": METRIC,
        "value": n / dt_b,
        "unit": "columns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt_b * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"cd2d {args.grid}x{args.grid} upwind convection-diffusion, convection U[-50,50]^2*h "
                               "seed 0 (n=%d, nnz=%d); RSAI(tol) c=3 lmax=8 eps=0.4 tol=1e-3" % (n, nnz),
                   "n": n, "nnz": nnz, "nnzM": int(nnzM), "schedule": "batched"},
        "roofline": {"bound": "alu", "achieved": achieved_tf, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved_tf / FP64_PEAK_TFLOPS, "traffic": measured_traffic(),
                     "kernel": "tier_kernel<8,3,12,6> (with the later size classes' launches)",
                     "kernel_ms": k_ms, "tier0_ms": t0_ms,
                     "basis": "model flops of every column / HIP-event time of all size-class kernels",
                     "alg_flops": flops, "hbm_alg_bytes": bytes_alg, "hbm_achieved_GBs": hbm_gbs,
                     "hbm_frac": hbm_gbs / HBM_PEAK_GBS, "measured_peaks": measured},
        "plain": plain,
        "speedup_vs_plain": (plain["ms_per_step"] / (dt_b * 1e3)) if plain else None,
        "graph_rebuild": graph,
        "fwd_bwd_ms": fwd_bwd_ms,
        "adjoint_roofline": adj_roof,
        "extra": extra,
        "build_event_ms": float(np.median(build_ms)),
        "phase_ms": {k: float(v) for k, v in t.items()},
        "cpu_baseline": cpu,
        # the paper's own construction timings, context only: n / ptime of its Tables 2
        # and 5 (collection matrices, n = 541 .. 21200), one core of the machine it names
        "paper_context": {"columns_per_s_range": [202, 14286], "kind": "n / ptime, Tables 2 and 5",
                          "hardware": "Intel Core 2 Quad E8400 3.0 GHz, 2 GB, Fortran 90, sequential"},
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
