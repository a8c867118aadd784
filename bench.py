#!/usr/bin/env python3
"""Benchmark of the spectral-element pressure-solve hot path on one MI355X.

Headline workload: 32^3 = 32,768 hexahedra at N = 7 (16,777,216 local
points) on the unit cube, vertices displaced by 0.05 h sin(2 pi .) sin(2 pi .),
homogeneous Dirichlet boundaries, Helmholtz h1 = 1, h2 = 0.1, right-hand side
from seeded Gaussian Fourier modes k <= 8.

One timed step = one application of the assembled operator: sem_ax (local
operator) followed by sem_dssum (gather-scatter + mask), FP64, inputs resident
in HBM.  `value` = local points x steps / wall time (GDOF/s).

Beside the headline (not in it): the time to a 1e-10 relative residual of
every solver form on the same GPU (FP64 Jacobi-PCG, the paper's restarted
GMRES with the hybrid Schwarz multigrid preconditioner, block-Jacobi CG,
defect correction, nested flexible CG, reliable updates) on the 32^3 mesh,
the 4^3 N = 5 manufactured-solution cube, the 16^3 channel (with the learned
smoother trained there) and the 64^3 channel; the FP64 CPU oracle timed on
the host cores.

roofline: the dominant kernel (the local operator) moves 72 algorithmic bytes
per local point (u, six geometric factors, B, w in FP64); achieved = 72 B x
n_local / its mean launch time from HIP events on the launch stream.
"""
import argparse
import ctypes
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
B_ALG_HELMHOLTZ_F64 = 72.0       # u, 6 G, B, w per local point (FP64)
B_DSSUM_SHARED_F64 = 16.0        # a shared local value read once and written once


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=200)
    p.add_argument("--warmup", type=int, default=10)
    p.add_argument("--solve-reps", type=int, default=3)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-solve", action="store_true")
    p.add_argument("--nel", type=int, default=32, help="elements per direction (32 = headline)")
    p.add_argument("--no-mixed", action="store_true", help="skip the FP32/BF16 refinement solves")
    p.add_argument("--no-learned", action="store_true", help="skip training and timing the learned smoother")
    p.add_argument("--no-large", action="store_true", help="skip the 64^3 channel workload")
    p.add_argument("--no-small", action="store_true", help="skip the 4^3 cube and 16^3 channel solves")
    p.add_argument("--train-fields", type=int, default=300,
                   help="16^3-channel right-hand sides generated online for training (2000 = the full set)")
    p.add_argument("--heldout", type=int, default=4)
    p.add_argument("--profile-kernels", action="store_true",
                   help="only launch the operator, gather-scatter and solver kernels a few times plus a "
                        "1 GiB torch copy (reference for hardware byte counters), then exit")
    return p.parse_args()


def stats(xs):
    """median and 95 % confidence half-width (normal approximation) of a sample."""
    med = statistics.median(xs)
    ci = 1.96 * statistics.stdev(xs) / math.sqrt(len(xs)) if len(xs) > 1 else 0.0
    return med, ci


def profile_kernels():
    """Short, fixed launch sequence for rocprofv3 counter runs on the 32^3
    workload: 5 x (sem_ax, sem_dssum) in FP64, 5 x sem_ax in FP32 and split
    BF16, a 300-iteration FP64 PCG solve, 300-iteration FP32 and BF16
    reliable-update solves, a 20-iteration GMRES with the multigrid
    preconditioner, and 5 copies of a 1 GiB buffer (exactly 1 GiB read + 1 GiB
    written each); then on the 16^3 channel 5 BF16 and 5 FP32 smoother
    applications, 5 training steps, 20 iterations of CG with the multigrid
    and 30 of flexible CG with the learned multigrid."""
    import numpy as np
    import torch

    from paper_2405_05640_amd import sem
    from paper_2405_05640_amd import workloads as wl
    torch.cuda.set_device(0)
    spec = wl.deformed_cube(32, 7)
    mesh = sem.Mesh.from_spec(spec, prepare=sem.SEM_PREP_F32 | sem.SEM_PREP_BF16 | sem.SEM_PREP_HSMG)
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
    x.zero_()
    mesh.pcg_solve(b, x, h1=1.0, h2=0.1, max_iter=20, raise_on_error=False, form=sem.FORM_GMRES_HSMG)
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    del mesh, u, w, u32, w32, b, x, src, dst
    torch.cuda.empty_cache()
    mesh = sem.Mesh.from_spec(wl.config("c3"), prepare=sem.SEM_PREP_HSMG)
    sm = sem.Smoother(mesh, seed=1)
    wts = sm.get_weights()
    wts[-432:] = np.random.default_rng(0).standard_normal(432).astype(np.float32) * 0.05
    sm.set_weights(wts)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(3)
    r = torch.randn(mesh.shape, dtype=torch.float64, device="cuda", generator=gen)
    mesh.dssum(r, mask=True)
    z = torch.empty_like(r)
    for fp32 in (False, True):
        for _ in range(5):
            sm.apply(r, z, fp32=fp32)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(5):
        sm.train_step(torch.randn(mesh.n_global, device="cuda", generator=gen), loss)
    x = torch.zeros_like(r)
    mesh.pcg_solve(r, x, max_iter=20, raise_on_error=False, form=sem.FORM_PCG_HSMG, check_every=4)
    x.zero_()
    zero = sem.Smoother(mesh, seed=1)   # zero last layer: no fallback, so every iteration runs the network
    mesh.pcg_solve(r, x, max_iter=30, raise_on_error=False, form=sem.FORM_FCG_LEARNED_MG, smoother=zero,
                   check_every=4)
    torch.cuda.synchronize()
    print("profile-kernels: done", flush=True)


def timed_solves(mesh, b, reps, **kw):
    """Median and 95 % CI of the wall time of `reps` solves from x = 0 (after
    one warm-up solve), with the last report."""
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
    med, ci = stats(times)
    del ws
    return {"median_ms": round(med, 3), "ci95_ms": round(ci, 3), "reps": reps, "iterations": rep.iterations,
            "outer_iterations": rep.outer_iterations, "true_rel_res": rep.true_rel_res,
            "fallback_used": rep.fallback_used}, x


def run_forms(mesh, b, forms, reps, ref_name="fp64_jacobi_pcg", tag=""):
    """Time every (name, kwargs) form on one mesh and right-hand side; adds
    the speed-up over the reference form and the distance of each solution
    to the reference solution."""
    import torch

    from paper_2405_05640_amd import sem
    out, xref, tref = {}, None, None
    for name, kw in forms:
        try:
            r, x = timed_solves(mesh, b, reps, **kw)
        except sem.SemError as exc:
            out[name] = {"status": "failed", "error": str(exc)}
            print("%s %s: %s" % (tag, name, exc), flush=True)
            continue
        if name == ref_name:
            xref, tref = x.clone(), r["median_ms"]
        elif xref is not None:
            r["rel_diff_vs_fp64_pcg"] = float(torch.linalg.norm(x - xref) / torch.linalg.norm(xref))
            r["speedup_vs_fp64_pcg"] = round(tref / r["median_ms"], 3)
        out[name] = r
        print("%s %s: %d iterations (%d outer), %.2f ms, true rel res %.2e" %
              (tag, name, r["iterations"], r["outer_iterations"], r["median_ms"], r["true_rel_res"]), flush=True)
        del x
    return out


def velocity_section(mesh, b0, spec):
    """The velocity solves' form on the c1 mesh: three Helmholtz fields (h1 = 1,
    h2 = 5, a velocity-like mass shift; right-hand sides b0 and two more
    Gaussian Fourier fields) with block-Jacobi CG, solved together by
    sem_pcg_solve_batched (one batched operator launch per iteration) and,
    for comparison, as three single solves."""
    import torch

    from paper_2405_05640_amd import sem
    from paper_2405_05640_amd import workloads as wl
    h1, h2 = 1.0, 5.0
    xyz = torch.from_numpy(mesh.export(sem.FIELD_XYZ)).cuda()
    B = torch.empty((3,) + tuple(b0.shape), dtype=torch.float64, device="cuda")
    B[0].copy_(b0)
    for c in (1, 2):
        f = wl.fourier_eval(wl.gaussian_fourier(wl.RHS_SEED["c1"] + c), xyz[0], xyz[1], xyz[2]).contiguous()
        mesh.rhs(f, B[c])
        del f
    del xyz
    X = torch.zeros_like(B)
    kw = dict(h1=h1, h2=h2, rel_tol=1e-10, form=sem.FORM_PCG_BLOCK_JACOBI, check_every=32)
    sem.pcg_solve_batched(mesh, B, X, **kw)
    X.zero_()
    torch.cuda.synchronize()
    t = time.perf_counter()
    reps = sem.pcg_solve_batched(mesh, B, X, **kw)
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t) * 1e3
    its, ts = [], 0.0
    for c in range(3):
        x = torch.zeros_like(B[c])
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = mesh.pcg_solve(B[c], x, **kw)
        torch.cuda.synchronize()
        ts += (time.perf_counter() - t) * 1e3
        its.append(r.iterations)
    out = {"fields": 3, "h1": h1, "h2": h2, "batched_ms": round(tb, 2),
           "batched_iterations": [r.iterations for r in reps],
           "true_rel_res_max": max(r.true_rel_res for r in reps),
           "three_single_solves_ms": round(ts, 2), "single_iterations": its,
           "speedup_vs_single_solves": round(ts / tb, 3)}
    print("velocity fields, block-Jacobi CG: batched %.1f ms (%s), three single solves %.1f ms" %
          (tb, out["batched_iterations"], ts), flush=True)
    del B, X
    return out


def copy_bandwidth():
    """Measured bandwidth of a plain 1 GiB device-to-device copy (read + write)."""
    import torch
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ts = []
    for _ in range(10):
        ev[0].record()
        dst.copy_(src)
        ev[1].record()
        torch.cuda.synchronize()
        ts.append(ev[0].elapsed_time(ev[1]))
    med = statistics.median(ts)
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * (1 << 30) / (med * 1e-3) / 1e9


def learned_section(args):
    """Train the smoother on the 16^3 channel with right-hand sides generated
    online (each field's Jacobi-PCG iterate errors are used once, in order),
    then time flexible CG with it against Jacobi-PCG on held-out fields.
    Two networks: the plain smoother (loss of M(r) alone), and one trained in
    the context of the learned multigrid (loss of M(r) + C(r), C the
    multigrid's middle and coarse levels), on the same errors plus two
    white-noise errors per field; the second is timed inside the learned
    multigrid against the same cycle with a zero network (Jacobi on the fine
    level)."""
    import numpy as np
    import torch

    from paper_2405_05640_amd import sem
    from paper_2405_05640_amd import workloads as wl

    spec = wl.config("c3")
    mesh = sem.Mesh.from_spec(spec, prepare=sem.SEM_PREP_HSMG)
    xyz = mesh.export(sem.FIELD_XYZ)
    vm = wl.kolmogorov_velocity(wl.RHS_SEED["c3"])

    def rhs(t):
        f = torch.from_numpy(wl.fourier_on_elements(wl.divergence_source(vm, t), xyz, (16, 16, 16))).cuda()
        b = torch.empty_like(f)
        mesh.rhs(f, b)
        return b

    iters = [1, 2, 4, 8]
    ws = mesh.workspace(mesh.solve_opts())

    def snapshot_errors(t):
        b = rhs(t)
        e = torch.zeros(len(iters) * mesh.n_global, dtype=torch.float64, device="cuda")
        sem.pcg_snapshots(mesh, b, iters, e, workspace=ws)
        return [e[q * mesh.n_global:(q + 1) * mesh.n_global] for q in range(len(iters))]

    glo = torch.from_numpy(mesh.export(sem.FIELD_GLO_NUM).ravel()).cuda()
    free = torch.ones(mesh.n_global, dtype=torch.float32, device="cuda")
    free[glo[torch.from_numpy(mesh.export(sem.FIELD_MASK).ravel()).cuda().bool()]] = 0.0
    gen = torch.Generator(device="cuda")
    gen.manual_seed(7)

    def noise():
        return (torch.randn(mesh.n_global, generator=gen, device="cuda") * free).contiguous()

    held_err = snapshot_errors(3000) + snapshot_errors(3001)
    b0 = rhs(2500)
    r0, _ = timed_solves(mesh, b0, 1)
    rate = (1e-10) ** (1.0 / max(r0["iterations"], 1))
    sm = sem.Smoother(mesh, seed=0, lr=1e-3, stall_window=25, stall_rate=rate)
    smg = sem.Smoother(mesh, seed=0, lr=1e-3, stall_window=25, stall_rate=rate, mg_context=True)
    zero = sem.Smoother(mesh, seed=0, stall_window=25, stall_rate=rate)   # zero last layer: Jacobi

    def held_loss(s):
        return float(np.mean([s.loss_grad(e[glo].reshape(mesh.shape).contiguous())[0] for e in held_err]))

    loss_jacobi, loss_jacobi_mg = held_loss(sm), held_loss(smg)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    losses, losses_mg, t_data, t_train, t_train_mg = [], [], 0.0, 0.0, 0.0
    for t in range(args.train_fields):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        errs = [e.float().contiguous() for e in snapshot_errors(t)]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for e in errs:
            sm.train_step(e, loss)
            losses.append(loss.clone())
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for e in errs + [noise(), noise()]:
            smg.train_step(e, loss)
            losses_mg.append(loss.clone())
        torch.cuda.synchronize()
        t_data += t1 - t0
        t_train += t2 - t1
        t_train_mg += time.perf_counter() - t2
        if (t + 1) % 100 == 0:
            print("learned: %d fields, data %.1f s, training %.1f + %.1f s" % (t + 1, t_data, t_train, t_train_mg),
                  flush=True)
    lv = torch.cat(losses).cpu().numpy() if losses else np.zeros(0)
    lvm = torch.cat(losses_mg).cpu().numpy() if losses_mg else np.zeros(0)
    nq, nqm = max(1, len(lv) // 4), max(1, len(lvm) // 4)
    loss_trained, loss_trained_mg = held_loss(sm), held_loss(smg)
    forms = [("jacobi_pcg", {}), ("fcg_learned", dict(form=sem.FORM_FCG_LEARNED, smoother=sm)),
             ("fcg_learned_mg_zero_net", dict(form=sem.FORM_FCG_LEARNED_MG, smoother=zero, check_every=4)),
             ("fcg_learned_mg", dict(form=sem.FORM_FCG_LEARNED_MG, smoother=smg, check_every=4)),
             ("gmres_learned_mg", dict(form=sem.FORM_GMRES_LEARNED_MG, smoother=smg, restart=10))]
    res = {name: [] for name, _ in forms}
    for h in range(args.heldout):
        b = rhs(2000 + h)
        for name, kw in forms:
            r, _ = timed_solves(mesh, b, 2, **kw)
            res[name].append(r)
    mean_ms = {name: statistics.mean(r["median_ms"] for r in rs) for name, rs in res.items()}
    out = {"workload": "16^3 tanh-stretched channel, N=7, periodic x/z, Poisson, k^-5/3 divergence RHS",
           "train_fields": args.train_fields, "pairs": args.train_fields * len(iters), "snapshot_iters": iters,
           "generation": "online: each field's pairs are generated, used for one Adam step each, and dropped",
           "loss_first_quarter": round(float(lv[:nq].mean()), 5) if len(lv) else None,
           "loss_last_quarter": round(float(lv[-nq:].mean()), 5) if len(lv) else None,
           "data_gen_s": round(t_data, 2), "train_s": round(t_train, 2),
           "train_ms_per_step": round(t_train / max(len(lv), 1) * 1e3, 3),
           "heldout_one_step_error": {"jacobi": round(loss_jacobi, 4), "trained": round(loss_trained, 4),
                                      "what": "A-norm error energy left after one smoother application, "
                                              "held-out Jacobi-PCG iterate errors"},
           "mg_context_training": {"pairs": len(lvm), "extra": "two white-noise errors per field",
                                   "loss_first_quarter": round(float(lvm[:nqm].mean()), 5) if len(lvm) else None,
                                   "loss_last_quarter": round(float(lvm[-nqm:].mean()), 5) if len(lvm) else None,
                                   "train_s": round(t_train_mg, 2),
                                   "heldout_one_step_error": {"zero_net": round(loss_jacobi_mg, 4),
                                                              "trained": round(loss_trained_mg, 4),
                                                              "what": "A-norm error energy left after one "
                                                                      "learned-multigrid application"}},
           "heldout": args.heldout}
    for name, rs in res.items():
        out[name] = {"median_ms": round(mean_ms[name], 3), "iterations": [r["iterations"] for r in rs],
                     "fallback_used": [r["fallback_used"] for r in rs],
                     "true_rel_res_max": max(r["true_rel_res"] for r in rs)}
        if name != "jacobi_pcg":
            out[name]["speedup_vs_jacobi_pcg"] = round(mean_ms["jacobi_pcg"] / mean_ms[name], 3)
    args.learned_weights = smg.get_weights()
    out["speedup_vs_jacobi_pcg"] = out["fcg_learned_mg"]["speedup_vs_jacobi_pcg"]
    out["speedup_vs_jacobi_pcg_plain_smoother"] = out["fcg_learned"]["speedup_vs_jacobi_pcg"]
    out["network_gain_in_multigrid"] = round(mean_ms["fcg_learned_mg_zero_net"] / mean_ms["fcg_learned_mg"], 3)
    return out


def channel_rhs(mesh, cfg, nel, t=0):
    import torch

    from paper_2405_05640_amd import sem
    from paper_2405_05640_amd import workloads as wl
    xyz = mesh.export(sem.FIELD_XYZ)
    vm = wl.kolmogorov_velocity(wl.RHS_SEED[cfg])
    f = torch.from_numpy(wl.fourier_on_elements(wl.divergence_source(vm, t), xyz, (nel, nel, nel))).cuda()
    del xyz
    b = torch.empty_like(f)
    mesh.rhs(f, b)
    return b


def small_section(args):
    """Time to 1e-10 on the 4^3 N = 5 manufactured-solution cube and on the
    16^3 channel (latency-bound sizes)."""
    import torch

    from paper_2405_05640_amd import sem
    from paper_2405_05640_amd import workloads as wl
    out = {}
    spec = wl.config("c0")
    mesh = sem.Mesh.from_spec(spec, prepare=sem.SEM_PREP_HSMG)
    xyz = torch.from_numpy(mesh.export(sem.FIELD_XYZ)).cuda()
    _, f = wl.manufactured(xyz[0], xyz[1], xyz[2])
    b = torch.empty_like(xyz[0].contiguous())
    mesh.rhs(f.contiguous(), b)
    forms = [("fp64_jacobi_pcg", dict(check_every=8)), ("gmres_hsmg", dict(form=sem.FORM_GMRES_HSMG, restart=10)),
             ("pcg_hsmg", dict(form=sem.FORM_PCG_HSMG, check_every=4)),
             ("pcg_1red", dict(form=sem.FORM_PCG_1RED, check_every=8))]
    out["c0_cube4_N5"] = run_forms(mesh, b, forms, 5, tag="c0")
    del mesh
    spec = wl.config("c3")
    mesh = sem.Mesh.from_spec(spec, prepare=sem.SEM_PREP_HSMG | sem.SEM_PREP_F32)
    b = channel_rhs(mesh, "c3", 16)
    forms = [("fp64_jacobi_pcg", dict(check_every=32)), ("gmres_hsmg", dict(form=sem.FORM_GMRES_HSMG, restart=10)),
             ("pcg_hsmg", dict(form=sem.FORM_PCG_HSMG, check_every=4)),
             ("reliable_fp32", dict(form=sem.FORM_RELIABLE_FP32, inner_tol=0.1, check_every=32))]
    out["c3_channel16_N7"] = run_forms(mesh, b, forms, 3, tag="c3")
    return out


def large_section(args, learned_weights=None):
    """64^3 channel (262,144 elements, N = 7, Poisson): Ax+dssum rate and time
    to 1e-10 of FP64 Jacobi-PCG, GMRES and CG with the multigrid
    preconditioner, the reliable-update FP32 and split-BF16 solvers, and
    flexible CG with the learned multigrid: a zero network, and the network
    trained in the multigrid context on the 16^3 channel (learned_weights:
    the per-element network is the same on any mesh of order 7)."""
    import torch

    from paper_2405_05640_amd import sem
    from paper_2405_05640_amd import workloads as wl
    spec = wl.config("c4")
    t0 = time.perf_counter()
    mesh = sem.Mesh.from_spec(spec, prepare=sem.SEM_PREP_F32 | sem.SEM_PREP_BF16 | sem.SEM_PREP_HSMG)
    t_setup = time.perf_counter() - t0
    print("large: setup %.1f s" % t_setup, flush=True)
    b = channel_rhs(mesh, "c4", 64)
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
    forms = [("fp64_jacobi_pcg", dict(check_every=32, max_iter=40000)),
             ("gmres_hsmg", dict(form=sem.FORM_GMRES_HSMG, restart=10, max_iter=2000)),
             ("pcg_hsmg", dict(form=sem.FORM_PCG_HSMG, check_every=4, max_iter=2000)),
             ("reliable_fp32", dict(form=sem.FORM_RELIABLE_FP32, inner_tol=0.1, check_every=32, max_iter=40000)),
             ("reliable_bf16split", dict(form=sem.FORM_RELIABLE_BF16, inner_tol=0.1, check_every=32,
                                         max_iter=40000))]
    smoothers = []
    if learned_weights is not None:
        zero = sem.Smoother(mesh, seed=0)   # zero last layer: Jacobi on the fine level
        trained = sem.Smoother(mesh, seed=0)
        trained.set_weights(learned_weights)
        smoothers = [zero, trained]
        forms += [("fcg_learned_mg_zero_net", dict(form=sem.FORM_FCG_LEARNED_MG, smoother=zero, check_every=4,
                                                   max_iter=4000)),
                  ("fcg_learned_mg", dict(form=sem.FORM_FCG_LEARNED_MG, smoother=trained, check_every=4,
                                          max_iter=4000))]
    res = run_forms(mesh, b, forms, 1, tag="large")
    del smoothers
    return {"workload": "64^3 tanh-stretched channel, N=7, periodic x/z, Poisson (134,217,728 local points)",
            "setup_s": round(t_setup, 1), "ax_dssum_gdofs": round(mesh.n_local / dt / 1e9, 2),
            "ax_dssum_us": round(dt * 1e6, 1),
            "ax_dssum_hbm_frac": round(64.0 * mesh.n_local / dt / 1e9 / PEAK_HBM_GBS, 4),
            "time_to_1e-10": res}


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


def _omp_threads(n):
    """Set the OpenMP thread count of the oracle's parallel regions."""
    try:
        ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(n))
    except OSError:
        pass


def cpu_baseline(spec, h1, h2):
    """The FP64 CPU oracle on the host cores: S u on the full headline mesh
    (all cores; one thread on a 4-element-thick slab), and Jacobi-PCG time to
    1e-10 on the 4^3 N = 5 cube (all cores and one thread) and on the 16^3
    channel (a timed 40-iteration sample scaled to the iteration count the
    oracle needs, labelled as such)."""
    import numpy as np

    import oracle
    from paper_2405_05640_amd import workloads as wl
    cores = len(os.sched_getaffinity(0))
    _omp_threads(cores)
    om = oracle.Mesh(spec.nelx, spec.nely, spec.nelz, spec.order, spec.vertices, spec.periodic, spec.dirichlet)
    rng = np.random.default_rng(0)
    u = rng.standard_normal(om.shape)
    om.apply_S(u, h1, h2)
    reps, t0 = 0, time.perf_counter()
    while reps < 3 or time.perf_counter() - t0 < 4.0:
        om.apply_S(u, h1, h2)
        reps += 1
    el = time.perf_counter() - t0
    full = om.nl * reps / el / 1e9
    del om, u
    detail = {}
    # one thread, slab of the same mesh
    _omp_threads(1)
    nz = 4
    om = oracle.Mesh(spec.nelx, spec.nely, nz, spec.order, spec.vertices[: nz + 1], spec.periodic, spec.dirichlet)
    u = rng.standard_normal(om.shape)
    t0 = time.perf_counter()
    for _ in range(2):
        om.apply_S(u, h1, h2)
    detail["ax_dssum_gdofs_1thread"] = round(om.nl * 2 / (time.perf_counter() - t0) / 1e9, 4)
    del om, u
    # Jacobi-PCG to 1e-10, 4^3 N = 5 cube
    c0 = wl.config("c0")
    oc = oracle.Mesh(c0.nelx, c0.nely, c0.nelz, c0.order, c0.vertices, c0.periodic, c0.dirichlet)
    _, f = wl.manufactured(*oc.xyz)
    b = oc.rhs(f)
    for th, key in ((cores, "c0_pcg_ms_all_cores"), (1, "c0_pcg_ms_1thread")):
        _omp_threads(th)
        oc.pcg(b)
        t0 = time.perf_counter()
        _, info = oc.pcg(b)
        detail[key] = round((time.perf_counter() - t0) * 1e3, 3)
    detail["c0_pcg_iterations"] = info["iterations"]
    # 16^3 channel: timed sample, scaled
    _omp_threads(cores)
    c3 = wl.config("c3")
    o3 = oracle.Mesh(c3.nelx, c3.nely, c3.nelz, c3.order, c3.vertices, c3.periodic, c3.dirichlet)
    b3 = o3.rhs(rng.standard_normal(o3.shape))
    t0 = time.perf_counter()
    _, i40 = o3.pcg(b3, tol=1e-30, max_iter=40)
    per_it = (time.perf_counter() - t0) / 40
    detail["c3_pcg_ms_per_iteration_all_cores"] = round(per_it * 1e3, 3)
    detail["c3_pcg_ms_extrapolated"] = {"value": round(per_it * 865 * 1e3, 1),
                                        "how": "40 timed oracle iterations x 865 (the GPU Jacobi-PCG iteration "
                                               "count on this channel), extrapolated"}
    return {"value": full, "unit": "GDOF/s", "cores": cores, "kind": "oracle",
            "sample": "FP64 oracle S u = mask(dssum(A_L u)) on the full 32^3 N=7 deformed mesh "
                      "(16.8 M local points), %d applications in %.1f s on %d threads" % (reps, el, cores),
            "detail": detail}


def main():
    args = parse()
    if args.profile_kernels:
        profile_kernels()
        return
    if args.gpus != 1:
        print("bench.py: the solver runs on one GPU only (no sharding or collectives); "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2405_05640_amd import sem
    from paper_2405_05640_amd import workloads as wl

    torch.cuda.set_device(0)
    spec = wl.deformed_cube(args.nel, 7)
    h1, h2 = wl.HELMHOLTZ["c1"]
    t_setup = time.perf_counter()
    prep = 0 if args.no_solve else (sem.SEM_PREP_HSMG | (0 if args.no_mixed else sem.SEM_PREP_F32 | sem.SEM_PREP_BF16))
    mesh = sem.Mesh.from_spec(spec, prepare=prep)
    xyz = torch.from_numpy(mesh.export(sem.FIELD_XYZ)).cuda()
    f = wl.fourier_eval(wl.gaussian_fourier(wl.RHS_SEED["c1"]), xyz[0], xyz[1], xyz[2]).contiguous()
    del xyz
    b = torch.empty_like(f)
    mesh.rhs(f, b)
    del f
    torch.cuda.synchronize()
    print("setup %.1f s: E=%d n_local=%d n_global=%d" % (time.perf_counter() - t_setup, mesh.E,
                                                         mesh.n_local, mesh.n_global), flush=True)
    u = b.clone()
    w = torch.empty_like(u)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        mesh.ax(u, w, h1, h2)
        mesh.dssum(w, mask=True)
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
    wall = time.perf_counter() - t0
    ax_ms = [ev[q][0].elapsed_time(ev[q][1]) for q in range(args.steps)]
    gs_ms = [ev[q][1].elapsed_time(ev[q][2]) for q in range(args.steps)]
    ax_med, ax_ci = stats(ax_ms)
    gs_med, gs_ci = stats(gs_ms)
    ax_mean = statistics.mean(ax_ms)
    t_step = wall / args.steps
    value = mesh.n_local * args.steps / wall / 1e9
    achieved = B_ALG_HELMHOLTZ_F64 * mesh.n_local / (ax_mean * 1e-3) / 1e9
    f_shared = mesh.info["n_shared_local"] / mesh.n_local
    gs_bytes = B_DSSUM_SHARED_F64 * f_shared * mesh.n_local
    headline_frac = B_ALG_HELMHOLTZ_F64 * mesh.n_local / t_step / 1e9 / PEAK_HBM_GBS
    print("Ax %.1f us (%.0f GB/s alg), dssum %.1f us, step %.1f us, headline %.3f of 8 TB/s" %
          (ax_med * 1e3, achieved, gs_med * 1e3, t_step * 1e6, headline_frac), flush=True)
    del u, w
    torch.cuda.empty_cache()
    copy_gbs = copy_bandwidth()
    tr = traffic_record(os.path.join(ROOT, "paper_2405_05640_amd", "csrc", "ax.hip"))

    out = {
        "metric": "Ax+dssum GDOF/s (% HBM roofline); time-to-1e-10 Poisson solve, learned vs PCG",
        "value": round(value, 3),
        "unit": "GDOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_step * 1e3, 5),
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
        "headline_hbm_frac": round(headline_frac, 4),
        "headline_hbm_frac_def": "72 B x n_local / (Ax+dssum wall time per step) / 8 TB/s; the gather-scatter's "
                                 "bytes are overhead, not credited",
        "headline_vs_copy_frac": round(B_ALG_HELMHOLTZ_F64 * mesh.n_local / t_step / 1e9 / copy_gbs, 4),
        "copy_kernel_gbs": round(copy_gbs, 1),
        "unique_node_rate_gdofs": round(mesh.n_global / t_step / 1e9, 3),
        "ax_launch_us": {"median": round(ax_med * 1e3, 2), "ci95": round(ax_ci * 1e3, 2)},
        "dssum_launch_us": {"median": round(gs_med * 1e3, 2), "ci95": round(gs_ci * 1e3, 2)},
        "dssum_roofline": {"bound": "hbm", "alg_bytes_per_point": round(B_DSSUM_SHARED_F64 * f_shared, 3),
                           "achieved": round(gs_bytes / (gs_med * 1e-3) / 1e9, 1), "peak": PEAK_HBM_GBS,
                           "unit": "GB/s", "frac": round(gs_bytes / (gs_med * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
                           "kernel": "gs_seg_kernel<double,MASK,G,SPL> (sem_dssum)",
                           "def": "16 B x shared local points (read once, written once) / median launch time"},
    }

    if not args.no_solve:
        forms = [("fp64_jacobi_pcg", dict(check_every=32)),
                 ("gmres_hsmg", dict(form=sem.FORM_GMRES_HSMG, restart=10)),
                 ("pcg_hsmg", dict(form=sem.FORM_PCG_HSMG, check_every=4)),
                 ("pcg_block_jacobi", dict(form=sem.FORM_PCG_BLOCK_JACOBI, check_every=32))]
        if not args.no_mixed:
            forms += [("dc_fp32", dict(form=sem.FORM_DC_FP32, inner_tol=1e-5, max_outer=60, check_every=32)),
                      ("dc_bf16", dict(form=sem.FORM_DC_BF16, inner_tol=1e-2, max_outer=60, check_every=32)),
                      ("fcg_inner_fp32", dict(form=sem.FORM_FCG_INNER_FP32, inner_iters=8, inner_tol=0.0)),
                      ("fcg_inner_bf16", dict(form=sem.FORM_FCG_INNER_BF16, inner_iters=8, inner_tol=0.0)),
                      ("reliable_fp32", dict(form=sem.FORM_RELIABLE_FP32, inner_tol=0.1, check_every=32)),
                      ("reliable_bf16split", dict(form=sem.FORM_RELIABLE_BF16, inner_tol=0.1, check_every=32))]
        forms = [(n, dict(kw, h1=h1, h2=h2, rel_tol=1e-10)) for n, kw in forms]
        out["time_to_1e-10_ms"] = run_forms(mesh, b, forms, args.solve_reps, tag="c1")
        out["velocity_batched_block_jacobi"] = velocity_section(mesh, b, spec)
    del mesh, b
    torch.cuda.empty_cache()
    if not args.no_small and not args.no_solve:
        out["small_configs"] = small_section(args)
        torch.cuda.empty_cache()
    if not args.no_learned:
        out["learned_smoother"] = learned_section(args)
        print("learned: %s" % json.dumps(out["learned_smoother"]), flush=True)
        torch.cuda.empty_cache()
    if not args.no_large and not args.no_solve:
        out["large_single_gpu"] = large_section(args, getattr(args, "learned_weights", None))
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(spec, h1, h2)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
