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
B_ALG_DSSUM_F64 = 16.0      # every local value read once and written once


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=200)
    p.add_argument("--warmup", type=int, default=10)
    p.add_argument("--solve-reps", type=int, default=3)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-solve", action="store_true")
    p.add_argument("--nel", type=int, default=32, help="elements per direction (32 = headline)")
    p.add_argument("--no-mixed", action="store_true", help="skip the FP32/BF16 defect-correction solves")
    p.add_argument("--no-learned", action="store_true", help="skip training and timing the learned smoother")
    p.add_argument("--train-fields", type=int, default=48, help="channel fields used for training pairs")
    p.add_argument("--train-epochs", type=int, default=4)
    p.add_argument("--heldout", type=int, default=4)
    p.add_argument("--large", action="store_true",
                   help="also run the 64^3 channel workload (134M local points): operator rate, FP64 "
                        "Jacobi-PCG and reliable-update FP32 / split-BF16 time to 1e-10")
    p.add_argument("--profile-kernels", action="store_true",
                   help="only launch the operator, gather-scatter and CG kernels a few times plus a "
                        "1 GiB torch copy (reference for hardware byte counters), then exit")
    return p.parse_args()


def profile_kernels():
    """Short, fixed launch sequence for rocprofv3 counter runs on the 32^3
    workload: 5 x (sem_ax, sem_dssum) in FP64, 5 x sem_ax in FP32 and split
    BF16, a 300-iteration FP64 PCG solve and 300-iteration FP32 and BF16
    reliable-update solves (the solvers' gather-mode kernels), and 5 copies of
    a 1 GiB buffer (exactly 1 GiB read + 1 GiB written each)."""
    import torch

    from paper_2405_05640_amd import sem
    from paper_2405_05640_amd import workloads as wl
    torch.cuda.set_device(0)
    spec = wl.deformed_cube(32, 7)
    mesh = sem.Mesh.from_spec(spec, prepare=sem.SEM_PREP_F32 | sem.SEM_PREP_BF16)
    u = torch.rand(mesh.shape, dtype=torch.float64, device="cuda")
    w = torch.empty_like(u)
    for _ in range(5):
        mesh.ax(u, w, 1.0, 0.1)
        mesh.dssum(w, mask=True)
    u32 = u.float()
    w32 = torch.empty_like(u32)
    for _ in range(5):
        mesh.ax(u32, w32, 1.0, 0.1, dtype=sem.SEM_F32)
    for _ in range(5):
        mesh.ax(u32, w32, 1.0, 0.1, dtype=sem.SEM_BF16_SPLIT)
    b = torch.empty_like(u)
    mesh.rhs(u, b)
    x = torch.zeros_like(b)
    mesh.pcg_solve(b, x, h1=1.0, h2=0.1, max_iter=300, raise_on_error=False)
    for form in (sem.FORM_RELIABLE_FP32, sem.FORM_RELIABLE_BF16):
        x.zero_()
        mesh.pcg_solve(b, x, h1=1.0, h2=0.1, max_iter=300, raise_on_error=False, form=form, inner_tol=0.1)
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print("profile-kernels: done", flush=True)


def timed_solves(mesh, b, reps, **kw):
    """Median wall time of `reps` solves from x = 0 (after one warm-up)."""
    import torch
    x = torch.zeros_like(b)
    ws = mesh.workspace(mesh.solve_opts(**kw))
    times, rep = [], None
    for q in range(reps + 1):
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rep = mesh.pcg_solve(b, x, workspace=ws, **kw)
        torch.cuda.synchronize()
        if q > 0:
            times.append((time.perf_counter() - t0) * 1e3)
    med = statistics.median(times)
    ci = 1.96 * statistics.stdev(times) / math.sqrt(len(times)) if len(times) > 1 else 0.0
    return {"median": round(med, 2), "ci95": round(ci, 2), "iterations": rep.iterations,
            "outer_iterations": rep.outer_iterations, "true_rel_res": rep.true_rel_res,
            "fallback_used": rep.fallback_used}, x


def learned_section(args):
    """Train the smoother on the 16^3 channel workload, then time flexible CG
    with it against Jacobi-PCG on held-out fields (same GPU, same process)."""
    import numpy as np
    import torch

    from paper_2405_05640_amd import sem
    from paper_2405_05640_amd import workloads as wl

    spec = wl.config("c3")
    mesh = sem.Mesh.from_spec(spec)
    xyz = mesh.export(sem.FIELD_XYZ)
    vm = wl.kolmogorov_velocity(wl.RHS_SEED["c3"])

    def rhs(t):
        f = torch.from_numpy(wl.fourier_on_elements(wl.divergence_source(vm, t), xyz, (16, 16, 16))).cuda()
        b = torch.empty_like(f)
        mesh.rhs(f, b)
        return b

    # training pairs: errors of early Jacobi-PCG iterates
    t0 = time.perf_counter()
    iters = [1, 2, 4, 8]
    ws = mesh.workspace(mesh.solve_opts())

    def snapshot_errors(ts):
        out = []
        for t in ts:
            b = rhs(t)
            e = torch.zeros(len(iters) * mesh.n_global, dtype=torch.float64, device="cuda")
            sem.pcg_snapshots(mesh, b, iters, e, workspace=ws)
            out += [e[q * mesh.n_global:(q + 1) * mesh.n_global].contiguous() for q in range(len(iters))]
        return out

    pairs = [e.float().contiguous() for e in snapshot_errors(range(args.train_fields))]
    held_err = snapshot_errors(range(3000, 3002))
    glo = torch.from_numpy(mesh.export(sem.FIELD_GLO_NUM).ravel()).cuda()
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    # Jacobi-PCG reference rate for the stall test
    b0 = rhs(args.train_fields + 1000)
    r0, _ = timed_solves(mesh, b0, 1)
    rate = (1e-10) ** (1.0 / max(r0["iterations"], 1))
    sm = sem.Smoother(mesh, seed=0, lr=1e-3, stall_window=25, stall_rate=rate)

    def held_loss():
        return float(np.mean([sm.loss_grad(e[glo].reshape(mesh.shape).contiguous())[0] for e in held_err]))

    loss_jacobi = held_loss()   # fresh smoother: zero last layer, exactly Jacobi
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    losses = []
    t0 = time.perf_counter()
    order = np.random.default_rng(0).permutation(len(pairs))
    for ep in range(args.train_epochs):
        acc = []
        for k in order:
            sm.train_step(pairs[k], loss)
            acc.append(loss)
            loss = torch.zeros(1, dtype=torch.float64, device="cuda")
        losses.append(float(torch.cat(acc).mean().item()))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    loss_trained = held_loss()
    del pairs
    # held-out fields (t beyond the training range)
    res_j, res_l = [], []
    for h in range(args.heldout):
        b = rhs(2000 + h)
        rj, _ = timed_solves(mesh, b, 2)
        rl, _ = timed_solves(mesh, b, 2, form=sem.FORM_FCG_LEARNED, smoother=sm)
        res_j.append(rj)
        res_l.append(rl)
    tj = statistics.mean(r["median"] for r in res_j)
    tl = statistics.mean(r["median"] for r in res_l)
    return {"workload": "16^3 tanh-stretched channel, N=7, periodic x/z, Poisson, k^-5/3 divergence RHS",
            "train_fields": args.train_fields, "pairs": args.train_fields * len(iters),
            "snapshot_iters": iters, "epochs": args.train_epochs, "loss_per_epoch": [round(v, 5) for v in losses],
            "data_gen_s": round(t_data, 2), "train_s": round(t_train, 2),
            "heldout_one_step_error": {"jacobi": round(loss_jacobi, 4), "trained": round(loss_trained, 4),
                                       "what": "A-norm error energy left after one smoother application, "
                                               "held-out Jacobi-PCG iterate errors"},
            "heldout": args.heldout,
            "jacobi_pcg": {"median_ms": round(tj, 2),
                           "iterations": [r["iterations"] for r in res_j]},
            "fcg_learned": {"median_ms": round(tl, 2), "iterations": [r["iterations"] for r in res_l],
                            "fallback_used": [r["fallback_used"] for r in res_l],
                            "true_rel_res_max": max(r["true_rel_res"] for r in res_l)},
            "speedup_vs_jacobi_pcg": round(tj / tl, 3)}


def large_section(args):
    """64^3 channel (262,144 elements, N = 7, Poisson): Ax+dssum rate and
    time to 1e-10 for FP64 Jacobi-PCG and the reliable-update FP32 and split
    BF16 solvers."""
    import torch

    from paper_2405_05640_amd import sem
    from paper_2405_05640_amd import workloads as wl
    spec = wl.config("c4")
    t0 = time.perf_counter()
    mesh = sem.Mesh.from_spec(spec, prepare=sem.SEM_PREP_F32 | sem.SEM_PREP_BF16)
    t_setup = time.perf_counter() - t0
    print("large: setup %.1f s" % t_setup, flush=True)
    xyz = mesh.export(sem.FIELD_XYZ)
    vm = wl.kolmogorov_velocity(wl.RHS_SEED["c4"])
    f = torch.from_numpy(wl.fourier_on_elements(wl.divergence_source(vm, 0), xyz, (64, 64, 64))).cuda()
    del xyz
    b = torch.empty_like(f)
    mesh.rhs(f, b)
    del f
    w = torch.empty_like(b)
    for _ in range(3):
        mesh.ax(b, w, 1.0, 0.0)
        mesh.dssum(w, mask=True)
    torch.cuda.synchronize()
    n = 10
    t0 = time.perf_counter()
    for _ in range(n):
        mesh.ax(b, w, 1.0, 0.0)
        mesh.dssum(w, mask=True)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / n
    del w
    print("large: Ax+dssum %.1f us" % (dt * 1e6), flush=True)
    r64, _ = timed_solves(mesh, b, 1, rel_tol=1e-10, check_every=32, max_iter=40000)
    print("large: FP64 PCG %s" % json.dumps(r64), flush=True)
    out = {"workload": "64^3 tanh-stretched channel, N=7, periodic x/z, Poisson (134,217,728 local points)",
           "setup_s": round(t_setup, 1), "ax_dssum_gdofs": round(mesh.n_local / dt / 1e9, 2),
           "ax_dssum_us": round(dt * 1e6, 1), "fp64_jacobi_pcg": r64}
    for name, form in (("reliable_fp32", sem.FORM_RELIABLE_FP32), ("reliable_bf16split", sem.FORM_RELIABLE_BF16)):
        try:
            rr, _ = timed_solves(mesh, b, 1, rel_tol=1e-10, check_every=32, max_iter=40000, form=form, inner_tol=0.1)
        except sem.SemError as exc:
            out[name] = {"status": "failed", "error": str(exc)}
            continue
        rr["speedup_vs_fp64_pcg"] = round(r64["median"] / rr["median"], 3)
        out[name] = rr
        print("large: %s %s" % (name, json.dumps(rr)), flush=True)
    return out


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
        if el >= budget_s:
            break
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    return {"value": om.nl * reps / el / 1e9, "unit": "GDOF/s", "cores": threads, "kind": "oracle",
            "sample": "FP64 oracle S u = mask(dssum(A_L u)) on a %dx%dx%d-element slab of the same "
                      "deformed mesh (N=%d, %d local points), %d applications in %.1f s"
                      % (spec.nelx, spec.nely, nz, spec.order, om.nl, reps, el)}


def main():
    args = parse()
    if args.profile_kernels:
        profile_kernels()
        return
    if args.gpus != 1:
        print("bench.py: the solver runs on one GPU only (no sharding or collectives); "
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
    gs_achieved = B_ALG_DSSUM_F64 * mesh.n_local / (gs_mean * 1e-3) / 1e9
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
                     "traffic": tr, "kernel": "ax_pt_kernel<double,8,HELM> (sem_ax local operator)",
                     "alg_bytes_per_point": B_ALG_HELMHOLTZ_F64,
                     "mean_launch_us": round(ax_mean * 1e3, 2)},
        "dssum_mean_us": round(gs_mean * 1e3, 2),
        "dssum_roofline": {"bound": "hbm", "achieved": round(gs_achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                           "frac": round(gs_achieved / PEAK_HBM_GBS, 4),
                           "kernel": "gs_seg_kernel<double,MASK,G,SPL> (sem_dssum)",
                           "alg_bytes_per_point": B_ALG_DSSUM_F64, "mean_launch_us": round(gs_mean * 1e3, 2)},
        "ax_dssum_hbm_frac": round((B_ALG_HELMHOLTZ_F64 + B_ALG_DSSUM_F64) * mesh.n_local / (wall / args.steps)
                                   / 1e9 / PEAK_HBM_GBS, 4),
    }

    if not args.no_solve:
        sol = {}
        r64, x64 = timed_solves(mesh, b, args.solve_reps, h1=h1, h2=h2, rel_tol=1e-10, check_every=32)
        r64["ms_per_iteration"] = round(r64["median"] / max(r64["iterations"], 1), 4)
        sol["fp64_jacobi_pcg"] = r64
        print("PCG: %d iterations, %.1f ms, true rel res %.2e" % (r64["iterations"], r64["median"],
                                                                r64["true_rel_res"]), flush=True)
        if not args.no_mixed:
            del mesh
            torch.cuda.empty_cache()
            mesh = sem.Mesh.from_spec(spec, prepare=sem.SEM_PREP_F32 | sem.SEM_PREP_BF16)
            forms = (("dc_fp32", sem.FORM_DC_FP32, 1e-5), ("dc_bf16", sem.FORM_DC_BF16, 1e-2),
                     ("fcg_inner_fp32", sem.FORM_FCG_INNER_FP32, 0.0), ("fcg_inner_bf16", sem.FORM_FCG_INNER_BF16, 0.0),
                     ("reliable_fp32", sem.FORM_RELIABLE_FP32, 0.1), ("reliable_bf16split", sem.FORM_RELIABLE_BF16, 0.1))
            for name, form, itol in forms:
                try:
                    rr, xx = timed_solves(mesh, b, args.solve_reps, h1=h1, h2=h2, rel_tol=1e-10, check_every=32,
                                          form=form, inner_tol=itol, max_outer=60, inner_iters=8)
                except sem.SemError as exc:
                    sol[name] = {"status": "failed", "error": str(exc), "inner_tol": itol}
                    print("%s: %s" % (name, exc), flush=True)
                    continue
                d = xx - x64
                rr["rel_diff_vs_fp64_pcg"] = float(torch.linalg.norm(d) / torch.linalg.norm(x64))
                rr["inner_tol"] = itol
                rr["speedup_vs_fp64_pcg"] = round(r64["median"] / rr["median"], 3)
                sol[name] = rr
                print("%s: %d inner / %d outer, %.1f ms, true rel res %.2e" %
                      (name, rr["iterations"], rr["outer_iterations"], rr["median"], rr["true_rel_res"]), flush=True)
        out["time_to_1e-10_ms"] = sol
    if args.large:
        del mesh, b
        torch.cuda.empty_cache()
        out["large_single_gpu"] = large_section(args)
        print("large: %s" % json.dumps(out["large_single_gpu"]), flush=True)
    if not args.no_learned:
        out["learned_smoother"] = learned_section(args)
        print("learned: %s" % json.dumps(out["learned_smoother"]), flush=True)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(spec, h1, h2)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
