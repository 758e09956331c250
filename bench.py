"""Benchmark: predictor-corrector time steps per second of the pipe-flow step.

Workload (default): N = 64 radial points, |m| < 48, |k| < 64 (3/2-dealiased
grid 64 x 144 x 192), alpha = 0.5, Re = 5300, dt = 0.005, fixed flux; a
synthetic state (laminar flow plus a seeded divergence-free perturbation of
10% of the laminar energy, broadband spectrum).  Inputs are resident in HBM
before the timed region.  One "step" is the whole hot path: two dealiased
nonlinear evaluations and two radial solves.

Prints one JSON line: headline value = FP64 steps/s; the mixed-precision form
(FP32 transforms and products, FP64 solves) is reported beside it, with the
roofline of the dominant kernel (HIP-event timed) and the CPU oracle timed on
this host.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
# The Newton-Krylov part runs three searches concurrently, one stream each;
# with HIP's default of 4 hardware queues per process two of their streams
# can land on one queue and serialise.  Set before HIP initialises.
os.environ.setdefault("GPU_MAX_HW_QUEUES", "8")

HBM_PEAK_GBS = 8000.0


def kernel_bytes(name, N, M, K, mixed):
    """Algorithmic bytes one launch moves: its inputs and outputs at the
    stored precision (per-unit figures times the units one launch covers)."""
    nk = 2 * K - 1
    cw = 8 if mixed else 16          # complex word of the transform path
    S64 = 16 * M * nk * N            # one FP64 spectral field
    S = cw * M * nk * N              # one spectral field in transform precision
    H = cw * N * M * 3 * K           # one z-transformed field
    if name == "zinv":
        return 6 * S + 6 * H
    if name == "theta":
        return 6 * H + 3 * H
    if name == "zfwd":
        return 3 * H + 3 * S
    if name == "solve_pred":   # read u^n, N^n; write u^p, omega^p
        return 3 * S64 + 3 * S + (6 * S if mixed else 6 * S64)
    if name == "solve_corr":   # read u^n, N^n, N^p; write u^{n+1}, omega (+ FP32 shadow)
        return 3 * S64 + 6 * S + 3 * S64 + (6 * S if mixed else 3 * S64)
    raise KeyError(name)


def solve_table_bytes(N, M, K, mp):
    """Operator tables one solve launch reads once besides the spectral
    fields, which the algorithmic count leaves out: the substitution images
    (8 NB + 32 doubles each, for N = NB) of the M K pressure and MU K
    Helmholtz operators, their 1/U_ii rows (NB doubles), the influence data
    (7 radial lines per (m, |k|)) and the 4 x 4 complex A^-1 per (m, k).
    None where N is not a padded row count (other image sizes)."""
    if N not in (32, 48, 64):
        return None
    MU, nk, NB = mp * (M - 1) + 2, 2 * K - 1, N
    return 8 * ((M + MU) * K * (8 * NB + 32 + NB) + M * K * 7 * N + M * nk * 32)


def step_bytes(N, M, K, mixed):
    """Bytes the step's kernels move: two nonlinear evaluations (with the
    z-transformed intermediate) and two solves."""
    return sum(kernel_bytes(k, N, M, K, mixed) * (2 if k in ("zinv", "theta", "zfwd") else 1)
               for k in ("zinv", "theta", "zfwd", "solve_pred", "solve_corr"))


def step_bytes_compulsory(N, M, K, mixed):
    """Transform-level compulsory bytes per step (spectral fields only): each
    nonlinear evaluation reads u, omega and writes N (9 fields), the
    predictor reads u^n, N^n and writes u^p, omega^p, the corrector reads
    u^n, N^n, N^p and writes u^{n+1}, omega."""
    nk = 2 * K - 1
    S64 = 16 * M * nk * N
    S = (8 if mixed else 16) * M * nk * N
    nl = 2 * 9 * S
    return nl + (3 * S64 + 3 * S + 6 * (S if mixed else S64)) + \
        (3 * S64 + 6 * S + 3 * S64 + (6 * S if mixed else 3 * S64))


def traffic_for(kernel, precision, workload):
    """HBM bytes per launch from the committed rocprofv3 counter summary of
    this workload, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}_{precision}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    src = os.path.join(ROOT, "paper_1705_03838_amd", "csrc", rec["source"])
    with open(src, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    if sha != rec.get("source_sha256"):
        return None
    return rec.get("hbm_bytes_per_launch")


def run_gpu(w, precision, steps, warmup, profile_steps, repeats=5):
    """Median over `repeats` timed runs of `steps` graph-launched steps (after
    `warmup` untimed ones), each bracketed by device synchronisation."""
    import torch

    import paper_1705_03838_amd as opf
    from inputs import workload_state

    s = opf.Solver(N=w["N"], M=w["M"], K=w["K"], mp=w["mp"], alpha=w["alpha"], Re=w["Re"],
                   dt=w["dt"], precision=precision)
    u0 = workload_state(w, s.nodes())
    s.set_state(torch.from_numpy(u0))
    s.step(warmup)
    times = []
    for _ in range(repeats):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(steps)
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) / steps)
    prof = s.profile_steps(profile_steps)
    diag = s.diagnostics(check=False)
    s.close()
    return float(np.median(times)), prof, diag, times


def run_adaptive(w, steps, warmup, courant=0.5, check_every=10, dt_max=0.01):
    """The pipe64 FP64 run under automatic time-step control (Courant limit;
    checks every `check_every` steps, each a CFL reduction plus the last
    correction, synchronising; a change rebuilds the dt tables on the host
    and recaptures the step graph)."""
    import torch

    import paper_1705_03838_amd as opf
    from inputs import workload_state

    s = opf.Solver(N=w["N"], M=w["M"], K=w["K"], mp=w["mp"], alpha=w["alpha"], Re=w["Re"],
                   dt=w["dt"], precision=opf.OPF_FP64)
    s.set_state(torch.from_numpy(workload_state(w, s.nodes())))
    s.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rep = s.step_adaptive(steps, courant=courant, pc_tol=0.0, dt_min=1e-5, dt_max=dt_max, grow=0.1,
                          check_every=check_every, trace=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    dts = rep["dts"]
    s.close()
    return {"steps": steps, "warmup_fixed_dt": warmup, "courant": courant, "check_every": check_every,
            "dt_max": dt_max, "wall_s": round(wall, 4), "steps_per_s": round(steps / wall, 2),
            "sim_time_per_s": round(rep["t"] / wall, 4), "checks": rep["checks"], "changes": rep["changes"],
            "rebuild_ms_total": round(rep["rebuild_ms"], 2),
            "rebuild_ms_per_change": round(rep["rebuild_ms"] / max(rep["changes"], 1), 2),
            "dt_first_last_min_max": [dts[0], dts[-1], min(dts), max(dts)],
            "cfl_last_check": rep["cfl"]}


def run_rotation(w, steps, warmup):
    """The pipe64 FP64 step with the Coriolis force of the paper's example
    (rotation axis perpendicular to the pipe, Ekman number 1): the theta
    kernel variant that adds -2 Omega x u at every dealiased point."""
    import torch

    import paper_1705_03838_amd as opf
    from inputs import workload_state

    om = 1.0 / (8.0 * 1.0 * w["Re"])  # E = nu / (2 Omega D^2) = 1
    s = opf.Solver(N=w["N"], M=w["M"], K=w["K"], mp=w["mp"], alpha=w["alpha"], Re=w["Re"], dt=w["dt"])
    s.set_rotation(om, 0.0, 0.0)
    s.set_state(torch.from_numpy(workload_state(w, s.nodes())))
    s.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps
    prof = s.profile_steps(20)
    s.close()
    return {"ekman": 1.0, "omega": om, "steps_per_s": round(1.0 / ms, 2), "ms_per_step": round(ms * 1e3, 4),
            "theta_us": round(prof["theta"][0] / max(prof["theta"][1], 1) * 1e3, 2)}


def record_krylov_pairs(w, seeds, gmres_m, shape):
    """Plain Newton-Krylov searches from the given seeds, run concurrently
    (one Solver and one HIP stream per search, one host thread each), every
    product J z recorded; returns the pairs concatenated in seed order, the
    wall time of the whole (contexts and buffers included), and each
    search's own wall time."""
    import threading

    import torch

    import paper_1705_03838_amd as opf
    from inputs import workload_state

    kw = dict(N=w["N"], M=w["M"], K=w["K"], mp=w["mp"], alpha=w["alpha"], Re=w["Re"], dt=w["dt"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solvers = [opf.Solver(stream=torch.cuda.Stream(), **kw) for _ in seeds]
    # device memory for each search (record buffer, Krylov workspace) taken
    # from its stream's pool here, so that the threads allocate nothing
    recs, xs = [], []
    for sv, seed in zip(solvers, seeds):
        with torch.cuda.stream(sv.stream):
            recs.append(torch.zeros((2 * gmres_m, 2) + tuple(shape), dtype=torch.complex128, device="cuda"))
            xs.append(torch.from_numpy(workload_state(dict(w, seed=seed), sv.nodes())).to("cuda"))
            torch.empty((gmres_m + 8) * 16 * int(np.prod(shape)), dtype=torch.uint8, device="cuda")
    out, errors = [None] * len(seeds), []

    def work(i, seed):
        s = solvers[i]
        try:
            with torch.cuda.stream(s.stream):
                t1 = time.perf_counter()
                _, r = s.nk_solve(xs[i], w["T"], 0.0, gmres_m=gmres_m, tol=1e-8, gmres_tol=1e-3, record=recs[i])
                s.stream.synchronize()
                out[i] = (recs[i][:r["recorded"]], round(time.perf_counter() - t1, 2))
        except Exception as e:  # re-raised below, in the calling thread
            errors.append(e)

    threads = [threading.Thread(target=work, args=(i, sd)) for i, sd in enumerate(seeds)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if errors:
        raise errors[0]
    pairs = torch.cat([o[0] for o in out])
    each = [o[1] for o in out]
    for s in solvers:
        s.close()
    return pairs, wall, each


def run_nk(w, gmres_m=40, probes=160, rank=16, train_steps=12000, batch=16, train_seeds=(5101, 5102, 5103),
           nonlaminar_energies=(1e-3,)):
    """Newton-Krylov travelling-wave search on the nk workload (N=48, |m|<24
    with 2-fold symmetry, |k|<32, Re 2400, alpha 1.25, T=20): seeded
    near-laminar guess (seed 5000), GMRES(40), tolerance 1e-8 on ||F||/||x||;
    first plain (restarted GMRES and a line search), then with the Krylov
    trust-region hookstep, then the Arnoldi stability of the solution found,
    then with the learned preconditioner trained two ways: on the (z, J z)
    pairs of the Krylov vectors that plain searches from other seeds
    (train_seeds) generate, and on Jacobian probes at laminar flow (run 32
    at a time as ensemble members).  Wall times are given for the search
    alone and with the training data and training included (both are made
    once per grid, Re and T and serve every later search).  Last, the same
    two networks at non-laminar base states: guesses of perturbation energy
    e (fractions of the laminar energy) for e in nonlaminar_energies."""
    import torch

    import paper_1705_03838_amd as opf
    from inputs import laminar_state, workload_state

    s = opf.Solver(N=w["N"], M=w["M"], K=w["K"], mp=w["mp"], alpha=w["alpha"], Re=w["Re"], dt=w["dt"])
    x0 = torch.from_numpy(workload_state(w, s.nodes()))

    def search(x=None, precond=None, hookstep=False, record=None, **kw):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xs, rep = s.nk_solve(x0 if x is None else x, w["T"], 0.0, gmres_m=gmres_m, tol=1e-8, gmres_tol=1e-3,
                             precond=precond, hookstep=hookstep, record=record, **kw)
        torch.cuda.synchronize()
        rep["wall_s"] = round(time.perf_counter() - t0, 3)
        rep["history"] = [float(f"{h:.3e}") for h in rep["history"]]
        search.last = xs
        return rep

    plain = search()
    # stability of the solution found: leading Floquet multipliers by Arnoldi
    v0 = torch.from_numpy(workload_state(dict(w, seed=w["seed"] + 1), s.nodes()) -
                          laminar_state(w["N"], w["M"], w["K"], s.nodes()))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev, arep = s.arnoldi(search.last, w["T"], 0.0, v0, m=40, nev=6, tol=1e-6, check_every=5)
    arn_s = time.perf_counter() - t0
    stability = {"products": arep["products"], "converged": arep["converged"], "wall_s": round(arn_s, 3),
                 "multipliers": [[float(f"{z.real:.6e}"), float(f"{z.imag:.6e}")] for z in ev],
                 "growth_rates": [float(f"{np.log(abs(z)) / w['T']:.6e}") for z in ev]}
    progress(f"nk arnoldi: {arep['products']} products, {arn_s:.1f} s")
    progress(f"nk plain: {plain['jvps']} jvps, {plain['wall_s']} s")
    hook = search(hookstep=True)
    progress(f"nk hookstep: {hook['jvps']} jvps, {hook['residual_evals']} residuals, {hook['wall_s']} s")
    # training data 1: the Krylov vectors of plain searches from other seeds
    # (every product recorded), the searches run concurrently, one context
    # and one stream each, from host threads (the library calls release the
    # GIL); each search alone is latency-bound on the nk grid
    krylov_pairs, krylov_s, krylov_sequential_s = record_krylov_pairs(w, train_seeds, gmres_m, s.shape)
    progress(f"nk krylov pairs: {krylov_pairs.shape[0]} from {len(train_seeds)} concurrent searches "
             f"in {krylov_s:.1f} s")
    # training data 2: Jacobian probes at laminar flow
    t0 = time.perf_counter()
    lam = torch.from_numpy(laminar_state(w["N"], w["M"], w["K"], s.nodes()))
    probe_pairs = s.probe_pairs(lam, w["T"], 0.0, probes, seed=11, batch=32)
    probe_s = time.perf_counter() - t0
    progress(f"nk probes: {probes} in {probe_s:.1f} s")

    def trained(pairs, data_s, label):
        net = opf.Mlp(s, width=256, layers=4, rank=rank, seed=3, lr=1e-3, lr_final=3e-5)
        t0 = time.perf_counter()
        losses = net.train_pairs(pairs, batch=batch, steps=train_steps, seed=5)
        train_s = time.perf_counter() - t0
        progress(f"nk training ({label}): {train_steps} steps in {train_s:.1f} s")
        pre = search(precond=net)
        flops_step = mlp_train_flops(net, s.M * (2 * s.K - 1))
        out = {"search": pre, "pairs": int(pairs.shape[0]), "data_s": round(data_s, 2),
               "train_steps": train_steps, "batch_pairs": batch, "lr": "cosine 1e-3 -> 3e-5",
               "train_s": round(train_s, 2), "train_step_ms": round(train_s / train_steps * 1e3, 4),
               "train_gemm_TFLOPs_lower_bound": round(flops_step * train_steps / train_s / 1e12, 2),
               "loss_first_last": [float(f"{losses[0]:.3e}"), float(f"{losses[-100:].mean():.3e}")],
               "wall_speedup_search": round(plain["wall_s"] / pre["wall_s"], 3),
               "wall_speedup_with_data_and_training": round(plain["wall_s"] / (pre["wall_s"] + data_s + train_s), 3),
               "jvp_ratio": round(plain["jvps"] / max(pre["jvps"], 1), 3),
               "break_even_searches": round((data_s + train_s) / max(plain["wall_s"] - pre["wall_s"], 1e-9), 2)}
        out["params"] = net.n_params
        return out, net

    krylov, knet = trained(krylov_pairs, krylov_s, "krylov")
    del krylov_pairs
    probed, pnet = trained(probe_pairs, probe_s, "probes")
    del probe_pairs
    # the same networks (trained near laminar flow) at non-laminar base states:
    # a guess of perturbation energy e (seed 5200), first Newton step and the
    # whole search (e <= 1e-3; larger e: first step only, up to 400 products)
    lam_norm = float(np.sqrt(s.vec_dot(lam, lam)))
    nonlaminar = []
    for e in nonlaminar_energies:
        xb = torch.from_numpy(workload_state(dict(w, seed=5200, energy_frac=e), s.nodes()))
        row = {"energy_frac": e, "seed": 5200}
        for label, net in (("plain", None), ("krylov", knet), ("probes", pnet)):
            first = search(xb, precond=net, max_newton=1, max_jvps=400)
            row[label] = {"first_step_products": first["jvps"], "first_step_fallbacks": first["fallbacks"],
                          "first_step_wall_s": first["wall_s"]}
            if e <= 1e-3:
                full = search(xb, precond=net)
                d = search.last - lam.to(search.last.device)
                row[label].update({"search": full, "distance_to_laminar": float(np.sqrt(s.vec_dot(d, d))) / lam_norm})
            progress(f"nk non-laminar E'={e:g} {label}: first step {first['jvps']} products")
        for label in ("krylov", "probes"):
            if "search" in row[label]:
                row[label]["wall_speedup_search"] = round(row["plain"]["search"]["wall_s"] / row[label]["search"]["wall_s"], 3)
        nonlaminar.append(row)
    knet.close()
    pnet.close()
    out = {"plain": plain, "hookstep": hook, "stability_arnoldi": stability,
           "steps_per_residual": int(round(w["T"] / w["dt"])),
           "network": {"width": 256, "layers": 4, "rank": rank, "params": krylov.pop("params")},
           "learned_krylov_pairs": dict(krylov, training_seeds=list(train_seeds), evaluation_seed=w["seed"],
                                        recording="concurrent searches, one stream each",
                                        recording_wall_s_each=krylov_sequential_s),
           "learned_laminar_probes": dict(probed, probe_batch=32, evaluation_seed=w["seed"]),
           "non_laminar_bases": nonlaminar}
    probed.pop("params", None)
    # the headline learned-preconditioner figures: Krylov-trained (the solver's own vectors)
    out["preconditioned"] = krylov["search"]
    out["wall_speedup"] = krylov["wall_speedup_search"]
    out["jvp_ratio"] = krylov["jvp_ratio"]
    s.close()
    return out


def profile_mlp(steps, rank=16):
    """Training-step timing of the learned preconditioner alone on the nk grid
    (for kernel traces): 32 random (z, J z) pairs of unit normals, batch 16,
    20 untimed steps, then `steps` timed steps."""
    import torch

    import paper_1705_03838_amd as opf
    from inputs import WORKLOADS

    w = WORKLOADS["nk"]
    s = opf.Solver(N=w["N"], M=w["M"], K=w["K"], mp=w["mp"], alpha=w["alpha"], Re=w["Re"], dt=w["dt"])
    g = torch.Generator(device="cpu").manual_seed(1)
    shape = (32, 2) + tuple(s.shape)
    pairs = torch.complex(torch.randn(shape, generator=g, dtype=torch.float64),
                          torch.randn(shape, generator=g, dtype=torch.float64)).cuda()
    net = opf.Mlp(s, width=256, layers=4, rank=rank)
    net.train_pairs(pairs, batch=16, steps=20)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    net.train_pairs(pairs, batch=16, steps=steps)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    flops = mlp_train_flops(net, s.M * (2 * s.K - 1))
    return {"mlp_train_step_ms": round(dt * 1e3, 4), "gemm_gflop_per_step": round(flops / 1e9, 2),
            "rank": rank, "steps": steps}


def mlp_train_flops(net, rows):
    """GEMM flops of one training step over the mode rows (padded to 32):
    forward 2 R (din H + L H^2 + H dout), backward twice that less the input
    gradient of the first layer."""
    rp = (rows + 31) // 32 * 32
    H, L, din, dout = net.width, net.layers, net.din, net.dout
    fwd = 2 * rp * (din * H + L * H * H + H * dout)
    bwd = 2 * rp * (din * H + 2 * L * H * H + 2 * H * dout)
    return fwd + bwd


def run_ensemble(steps=500, warmup=5):
    """96 independent trajectories in three resolution classes (32 x N=32,
    |m|<16, |k|<24; 32 x N=48, |m|<24, |k|<32; 32 x N=64, |m|<32, |k|<48),
    Re ~ U[1800, 2600], alpha ~ U[0.8, 1.6], perturbation energy log-uniform
    in [1e-4, 1e-1], mixed precision, one graph launch per step; the radial
    solve tile of each class chosen by the autotuner."""
    import torch

    import paper_1705_03838_amd as opf
    from inputs import ensemble_members, make_state

    mem = ensemble_members()
    kws = [dict(N=m["N"], M=m["M"], K=m["K"], mp=m["mp"], alpha=m["alpha"], Re=m["Re"], dt=m["dt"],
                precision=opf.OPF_MIXED) for m in mem]
    e = opf.Ensemble(kws)
    states = [make_state(m["N"], m["M"], m["K"], m["mp"], m["alpha"], e.members[i].nodes(),
                         m["energy_frac"], m["decay_m"], m["decay_k"], m["seed"], axis_power=1)
              for i, m in enumerate(mem)]
    for i, st in enumerate(states):
        e.members[i].set_state(torch.from_numpy(st))
    tune = e.tune(5)
    for i, st in enumerate(states):
        e.members[i].set_state(torch.from_numpy(st))
    e.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e.step(steps)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    finite = all(np.isfinite(e.members[i].diagnostics(check=False)["E"]) for i in (0, 32, 64))
    e.close()
    return {"members": len(mem), "steps": steps, "ms_per_step": round(dt * 1e3, 4),
            "member_steps_per_s": round(len(mem) / dt, 1), "precision": "mixed",
            "finite_after_run": finite, "autotune": tune}


def host_cpu():
    """Host CPU model and counts (the oracle's hardware)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable}


def cpu_baseline(w, nsteps=10):
    """The oracle as it stands, on this host: one untimed step to build its
    caches, then nsteps timed steps of the same workload from the same
    initial state.  The oracle's states after 0 and nsteps steps also give
    the accuracy of both GPU forms after nsteps steps, run on the oracle's
    radial nodes."""
    import torch
    from threadpoolctl import threadpool_info

    import paper_1705_03838_amd as opf
    from inputs import laminar_state, workload_state
    from oracle import Oracle, Params

    o = Oracle(Params(N=w["N"], M=w["M"], K=w["K"], mp=w["mp"], alpha=w["alpha"], Re=w["Re"],
                      dt=w["dt"]))
    r = o.g.r
    u0 = workload_state(w, r)
    o.step(u0)
    t0 = time.perf_counter()
    u = u0
    for _ in range(nsteps):
        u = o.step(u)
    dt = time.perf_counter() - t0
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    base = {"value": nsteps / dt, "unit": "steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{nsteps} FP64 predictor-corrector steps of the same workload from its initial "
                      f"state after one untimed step; {dt:.1f} s (numpy FFTs + LAPACK dense solves, "
                      f"{threads} BLAS threads)", **host_cpu()}
    lam = laminar_state(w["N"], w["M"], w["K"], r)
    acc = {}
    for name, prec in (("fp64", opf.OPF_FP64), ("mixed", opf.OPF_MIXED)):
        s = opf.Solver(N=w["N"], M=w["M"], K=w["K"], mp=w["mp"], alpha=w["alpha"], Re=w["Re"],
                       dt=w["dt"], precision=prec, r_nodes=r)
        s.set_state(torch.from_numpy(u0))
        s.step(nsteps)
        got = s.get_state().cpu().numpy()
        d = s.diagnostics(check=False)
        s.close()
        dref = o.diagnostics(u)
        e = o.energy_norm(got - u)
        acc[name] = {"velocity_rel": float(f"{e / o.energy_norm(u):.3e}"),
                     "velocity_rel_perturbation": float(f"{e / o.energy_norm(u - lam):.3e}"),
                     "energy_rel": float(f"{abs(d['E'] - dref['E']) / dref['E']:.3e}"),
                     "wall_shear_rel": float(f"{abs(d['tau_w'] - dref['tau_w']) / dref['tau_w']:.3e}"),
                     "max_coeff_rel": float(f"{np.max(np.abs(got - u)) / np.max(np.abs(u)):.3e}")}
    return base, {"steps": nsteps, "against": "FP64 oracle from the same initial state", **acc}


def progress(msg):
    """One line per finished phase on stderr (stdout carries only the JSON line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--profile-steps", type=int, default=100)
    ap.add_argument("--workload", default="pipe64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--fp64-only", action="store_true")
    ap.add_argument("--no-nk", action="store_true", help="skip the Newton-Krylov search")
    ap.add_argument("--nk-energies", default="1e-3",
                    help="comma-separated perturbation energies (fractions of laminar) of the non-laminar "
                         "base states the learned preconditioner is evaluated at")
    ap.add_argument("--no-ensemble", action="store_true", help="skip the 96-member ensemble")
    ap.add_argument("--no-adaptive", action="store_true", help="skip the run under time-step control")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run two plain 256 MiB copies, the runtime's device-to-device copy and "
                         "an elementwise one (known byte counts for scaling HBM counters)")
    ap.add_argument("--profile-mlp", type=int, default=0, metavar="STEPS",
                    help="only time STEPS training steps of the learned preconditioner (kernel traces)")
    args = ap.parse_args()
    if args.profile_mlp:
        print(json.dumps(profile_mlp(args.profile_mlp)), flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(ensemble members and Newton seeds would shard as independent units)", file=sys.stderr)
        sys.exit(2)

    import paper_1705_03838_amd as opf
    from inputs import WORKLOADS

    w = WORKLOADS[args.workload]
    N, M, K = w["N"], w["M"], w["K"]
    if args.calibrate_copy:
        # Two plain copies of 256 MiB for the byte counters: the runtime's
        # device-to-device copy (its blit kernel) and an elementwise kernel
        # (dst = src * 1) that reads through ordinary cached loads, as the
        # solver's kernels do.
        import torch
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    ms64, prof64, diag64, reps64 = run_gpu(w, opf.OPF_FP64, args.steps, args.warmup, args.profile_steps)
    progress(f"fp64 {args.workload}: {ms64 * 1e3:.4f} ms/step (median of {len(reps64)})")

    def roofline(prof, mixed, prec):
        """Dominant kernel by device time per step.  The predictor and
        corrector launches are one kernel (k_solve): its bytes per launch are
        the mean of the two launch kinds."""
        per = {k: (t / n if n else 0.0) for k, (t, n) in prof.items()}
        groups = {"zinv": ["zinv"], "theta": ["theta"], "zfwd": ["zfwd"],
                  "solve": ["solve_pred", "solve_corr"]}
        tot = {g: sum(prof[k][0] for k in ks) for g, ks in groups.items()}
        dom = max(tot, key=tot.get)
        ks = groups[dom]
        launches = sum(prof[k][1] for k in ks)
        bytes_all = sum(kernel_bytes(k, N, M, K, mixed) * prof[k][1] for k in ks)
        b = bytes_all / launches
        avg_ms = tot[dom] / launches
        ach = b / (avg_ms * 1e-3) / 1e9
        tr = traffic_for(dom, prec, args.workload)
        extra = {}
        tab = solve_table_bytes(N, M, K, w["mp"]) if dom == "solve" else None
        if tab is not None:  # the solve's traffic also holds its operator tables
            extra = {"tables_bytes_per_launch": tab,
                     "achieved_with_tables": round((b + tab) / (avg_ms * 1e-3) / 1e9, 1)}
        return {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                "traffic": tr, "alg_bytes_per_launch": int(b), **extra,
                "avg_launch_us": round(avg_ms * 1e3, 2),
                "kernels_us": {k: round(v * 1e3, 2) for k, v in per.items()}}

    out = {
        "metric": f"time steps/s (FP64 predictor-corrector step) and HBM GB/s at N={N}, |m|<{M}, |k|<{K}",
        "value": round(1.0 / ms64, 2),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms64 * 1e3, 4),
        "repeats_ms_per_step": [round(t * 1e3, 4) for t in reps64],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": f"synthetic: laminar pipe flow + seeded divergence-free perturbation "
                f"({100 * w['energy_frac']:g}% laminar energy)",
        "config": {"workload": f"{args.workload}: N={N} radial points, |m|<{M}, |k|<{K} "
                               f"(grid {N}x{3 * M}x{3 * K}), alpha={w['alpha']}, Re={w['Re']}, "
                               f"dt={w['dt']}, fixed flux, seed {w['seed']}",
                   "parallelism": "single GPU"},
        "alg_GBps_per_step": round(step_bytes_compulsory(N, M, K, False) / ms64 / 1e9, 1),
        "kernel_GBps_per_step": round(step_bytes(N, M, K, False) / ms64 / 1e9, 1),
        "roofline": roofline(prof64, False, "fp64"),
        "diagnostics_after_run": {k: diag64[k] for k in ("E", "D", "tau_w", "beta", "g_norm", "div_max", "cfl")},
    }
    if not args.fp64_only:
        ms32, prof32, _, reps32 = run_gpu(w, opf.OPF_MIXED, args.steps, args.warmup, args.profile_steps)
        progress(f"mixed {args.workload}: {ms32 * 1e3:.4f} ms/step")
        out["mixed"] = {"steps_per_s": round(1.0 / ms32, 2), "ms_per_step": round(ms32 * 1e3, 4),
                        "repeats_ms_per_step": [round(t * 1e3, 4) for t in reps32],
                        "speedup_vs_fp64": round(ms64 / ms32, 3),
                        "alg_GBps_per_step": round(step_bytes_compulsory(N, M, K, True) / ms32 / 1e9, 1),
                        "kernel_GBps_per_step": round(step_bytes(N, M, K, True) / ms32 / 1e9, 1),
                        "roofline": roofline(prof32, True, "mixed")}
    if not args.no_adaptive:
        out["coriolis"] = run_rotation(w, args.steps, args.warmup)
        progress(f"coriolis: {out['coriolis']['steps_per_s']} steps/s")
        ad = run_adaptive(w, args.steps, args.warmup)
        ad["fixed_dt_steps_per_s"] = out["value"]
        ad["fixed_dt_sim_time_per_s"] = round(w["dt"] / ms64, 4)
        out["adaptive_dt"] = ad
        progress(f"adaptive dt: {ad['steps_per_s']} steps/s, {ad['changes']} changes")
    if not args.no_ensemble:
        out["ensemble"] = run_ensemble()
        progress(f"ensemble: {out['ensemble']['ms_per_step']} ms/step")
    if not args.no_nk:
        out["newton_krylov"] = {"workload": "nk: N=48, |m|<24 (mp=2), |k|<32, alpha=1.25, Re=2400, "
                                            "dt=0.01, T=20, near-laminar seed 5000",
                                **run_nk(WORKLOADS["nk"], nonlaminar_energies=tuple(
                                    float(v) for v in args.nk_energies.split(",") if v))}
    if not args.no_cpu_baseline:
        out["cpu_baseline"], out["accuracy"] = cpu_baseline(w)
        progress(f"cpu baseline done; accuracy after {out['accuracy']['steps']} steps: "
                 f"fp64 {out['accuracy']['fp64']['velocity_rel']:.2e}, "
                 f"mixed {out['accuracy']['mixed']['velocity_rel']:.2e}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
