#!/usr/bin/env python3
"""Benchmark of the spectral-element pressure-solve hot path on one MI355X.

Workload (the headline configuration): 32^3 = 32,768 hexahedra at N = 7
(16,777,216 local points) on the unit cube, vertices displaced by
0.05 h sin(2 pi .) sin(2 pi .), homogeneous Dirichlet boundaries, Helmholtz
h1 = 1, h2 = 0.1, right-hand side from seeded Gaussian Fourier modes k <= 8.

One timed step = one application of the assembled operator: sem_ax (local
operator) followed by sem_dssum (gather-scatter + mask), FP64, inputs resident
in HBM.  `value` = local points x steps / wall time (GDOF/s).  After the
timed region the FP64 Jacobi-PCG time to a 1e-10 relative residual is
measured on the same workload (reported beside the headline, not in it).

roofline: the dominant kernel (the local operator) moves 72 algorithmic bytes
per local point (u, six geometric factors, B, w in FP64); achieved = 72 B x
n_local / its mean launch time from HIP events on the launch stream.
cpu_baseline: the FP64 CPU oracle on a bounded slab of the same mesh.
"""
import argparse
import hashlib
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
B_ALG_HELMHOLTZ_F64 = 72.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=200)
    p.add_argument("--warmup", type=int, default=10)
    p.add_argument("--solve-reps", type=int, default=3)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-solve", action="store_true")
    p.add_argument("--nel", type=int, default=32, help="elements per direction (32 = headline)")
    return p.parse_args()


def traffic_record(kernel_src):
    """HBM bytes per launch from committed rocprofv3 --pmc counters, only if
    they were taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "ax_f64_c1_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256(open(kernel_src, "rb").read()).hexdigest()
    if rec.get("kernel_sha256") != h:
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(spec, h1, h2, budget_s=12.0):
    """Oracle Ax+dssum+mask on a slab of the same mesh (nel x nel x 4 elements)."""
    import numpy as np

    import oracle
    nz = 4
    v = spec.vertices[: nz + 1]
    om = oracle.Mesh(spec.nelx, spec.nely, nz, spec.order, v, spec.periodic, spec.dirichlet)
    rng = np.random.default_rng(0)
    u = rng.standard_normal(om.shape)
    om.apply_S(u, h1, h2)
    reps, t0 = 0, time.perf_counter()
    while True:
        om.apply_S(u, h1, h2)
        reps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or reps >= 50:
            break
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    return {"value": om.nl * reps / el / 1e9, "unit": "GDOF/s", "cores": threads, "kind": "oracle",
            "sample": "FP64 oracle S u = mask(dssum(A_L u)) on a %dx%dx%d-element slab of the same "
                      "deformed mesh (N=%d, %d local points), %d applications in %.1f s"
                      % (spec.nelx, spec.nely, nz, spec.order, om.nl, reps, el)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (no sharding or collectives); "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2405_05640_amd import sem
    from paper_2405_05640_amd import workloads as wl

    torch.cuda.set_device(0)
    spec = wl.deformed_cube(args.nel, 7)
    h1, h2 = wl.HELMHOLTZ["c1"]
    t_setup = time.perf_counter()
    mesh = sem.Mesh.from_spec(spec)
    xyz = torch.from_numpy(mesh.export(sem.FIELD_XYZ)).cuda()
    f = wl.fourier_eval(wl.gaussian_fourier(wl.RHS_SEED["c1"]), xyz[0], xyz[1], xyz[2]).contiguous()
    del xyz
    b = torch.empty_like(f)
    mesh.rhs(f, b)
    torch.cuda.synchronize()
    print("setup %.1f s: E=%d n_local=%d n_global=%d" % (time.perf_counter() - t_setup, mesh.E,
                                                         mesh.n_local, mesh.n_global), flush=True)
    u = b.clone()
    w = torch.empty_like(u)
    stream = torch.cuda.current_stream()

    def step():
        mesh.ax(u, w, h1, h2)
        mesh.dssum(w, mask=True)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for q in range(args.steps):
        ev[q][0].record(stream)
        mesh.ax(u, w, h1, h2)
        ev[q][1].record(stream)
        mesh.dssum(w, mask=True)
        ev[q][2].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    ax_ms = [ev[q][0].elapsed_time(ev[q][1]) for q in range(args.steps)]
    gs_ms = [ev[q][1].elapsed_time(ev[q][2]) for q in range(args.steps)]
    ax_mean = statistics.mean(ax_ms)
    gs_mean = statistics.mean(gs_ms)
    value = mesh.n_local * args.steps / wall / 1e9
    achieved = B_ALG_HELMHOLTZ_F64 * mesh.n_local / (ax_mean * 1e-3) / 1e9
    print("Ax %.1f us (%.0f GB/s alg), dssum %.1f us, step %.1f us" %
          (ax_mean * 1e3, achieved, gs_mean * 1e3, wall / args.steps * 1e6), flush=True)
    tr = traffic_record(os.path.join(ROOT, "paper_2405_05640_amd", "csrc", "ax.hip"))

    out = {
        "metric": "Ax+dssum GDOF/s (% HBM roofline); time-to-1e-10 Poisson solve, learned vs PCG",
        "value": round(value, 3),
        "unit": "GDOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded deformed-cube mesh and Gaussian Fourier RHS)",
        "config": {"workload": "32^3 hex deformed cube, N=7, Helmholtz h1=1 h2=0.1, Dirichlet, FP64 "
                               "Ax+dssum" if args.nel == 32 else "%d^3 deformed cube N=7" % args.nel,
                   "elements": mesh.E, "order": 7, "n_local": mesh.n_local, "n_global": mesh.n_global,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": tr, "kernel": "ax_kernel<double,8,HELM> (local operator)",
                     "alg_bytes_per_point": B_ALG_HELMHOLTZ_F64,
                     "mean_launch_us": round(ax_mean * 1e3, 2)},
        "dssum_mean_us": round(gs_mean * 1e3, 2),
        "ax_dssum_hbm_frac": round(B_ALG_HELMHOLTZ_F64 * mesh.n_local / (wall / args.steps) / 1e9
                                   / PEAK_HBM_GBS, 4),
    }

    if not args.no_solve:
        times, its, rel = [], [], []
        x = torch.zeros_like(b)
        ws = mesh.workspace(mesh.solve_opts(h1=h1, h2=h2))
        for rep in range(args.solve_reps + 1):
            x.zero_()
            torch.cuda.synchronize()
            ts = time.perf_counter()
            r = mesh.pcg_solve(b, x, workspace=ws, h1=h1, h2=h2, rel_tol=1e-10, check_every=32)
            torch.cuda.synchronize()
            te = time.perf_counter()
            if rep > 0:
                times.append((te - ts) * 1e3)
                its.append(r.iterations)
                rel.append(r.true_rel_res)
        med = statistics.median(times)
        ci = 1.96 * statistics.stdev(times) / math.sqrt(len(times)) if len(times) > 1 else 0.0
        out["time_to_1e-10_ms"] = {"fp64_jacobi_pcg": {"median": round(med, 2), "ci95": round(ci, 2),
                                                       "iterations": its[0], "true_rel_res": rel[0],
                                                       "ms_per_iteration": round(med / its[0], 4)}}
        print("PCG: %d iterations, %.1f ms (%.1f us/iter), true rel res %.2e" %
              (its[0], med, med / its[0] * 1e3, rel[0]), flush=True)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(spec, h1, h2)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
