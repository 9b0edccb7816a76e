#!/usr/bin/env python3
"""Benchmark of the shared-Jacobian, frequency-shifted block solve on one MI355X.

Default workload (the largest single-GPU configuration): a three-row sector (rotor-
stator-rotor, 3 x 100x64x100 = 1,920,000 cells, 5,717,200 faces, pitch-overlap interfaces
between the rows), mean flow + 10 harmonics at mixed per-row frequencies, one Jacobian
stored in FP32 for all 11 systems.  One step is the whole hot path on inputs already
resident in HBM:
    assemble K from the FP64 state (Rusanov first-order Jacobian, eps = 0.6, sigma = 50)
    -> set the harmonics (factor slots invalidated) -> DILU factorisation of 11 systems
    -> preconditioned Richardson of all 11 systems to a 1e-8 relative residual drop,
       FP32 sweeps inside an FP64 defect correction with the exact FP64 operator.
Mesh ingest (validation, colouring, numbering: host work done once per mesh) is outside
the step and reported as ingest_ms.  Other workloads (--workload): the 200k-cell precision
configuration, 64 batched instances, the learned preconditioner's held-out protocol,
phase-lagged cascade, FGMRES, the RK driver, partitions.

value = cell-system-sweep updates per second: one update is the 6 complex unknowns of one
cell of one system advanced by one preconditioned sweep (x6 for scalar unknowns).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "cell-unknown updates/s; time to 1e-8 residual drop, plain vs learned+batched"
HBM_PEAK_GBS = 8000.0
SHAPE = (80, 50, 50)
N_HARM = 3
RTOL = 1e-8
CONVERGED = (0, 3)  # FNLH_OK, FNLH_FELL_BACK (learned corrections switched off, plain sweeps converged)
STATS_PERIOD = 4  # time the sweep-pass launches of every 4th sweep (bounds event overhead)


def build_inputs(shape=SHAPE):
    import numpy as np
    from paper_2404_01407_amd import synth
    mesh = synth.passage_block(*shape, 36, seed=2)
    Q = synth.flow_state(mesh, 2)
    om = synth.omegas_single_zone(N_HARM, 36)
    bs = [synth.rhs(mesh.n_cells, s, real=(s == 0)) for s in range(N_HARM + 1)]
    return mesh, Q, om, bs


class Runner:
    def __init__(self, mesh, Q, om, bs, storage, lanes=0, row_lanes=0, check_every=16, use_graph=True,
                 wave_groups=None):
        import torch
        from paper_2404_01407_amd import fnlh
        t0 = time.perf_counter()
        self.ctx = fnlh.Context(mesh, storage=storage, outer="exact")
        self.ingest_ms = 1e3 * (time.perf_counter() - t0)
        self.ctx.tune(sys_per_lane=lanes, lanes_per_row=row_lanes, wave_groups=wave_groups)
        self.check_every = check_every
        self.use_graph = use_graph
        self.Qd = torch.from_numpy(Q).cuda()
        self.bd = [torch.from_numpy(b).cuda() for b in bs]
        self.xd = [torch.zeros_like(b) for b in self.bd]
        self.om = om
        self.S = len(bs)
        self.N = mesh.n_cells

    def step(self):
        for x in self.xd:
            x.zero_()
        self.ctx.assemble_jacobian(self.Qd, eps=0.6, sigma=50.0)
        self.ctx.set_harmonics(self.om)
        st, rep = self.ctx.relax(list(range(self.S)), self.xd, self.bd, kind="dilu", max_sweeps=4000, rtol=RTOL,
                                 check_every=self.check_every, use_graph=self.use_graph)
        if st not in CONVERGED:
            raise RuntimeError(f"solve did not converge: status {st}, reports {rep}")
        return rep

    def timed(self, steps, warmup, stats=False):
        import torch
        for _ in range(warmup):
            self.step()
        if stats:
            self.ctx.stats_enable(True, period=STATS_PERIOD)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = []
        for _ in range(steps):
            reps.append(self.step())
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = self.ctx.stats() if stats else None
        if stats:
            self.ctx.stats_enable(False)
        updates = sum(self.N * r["sweeps"] for rep in reps for r in rep)
        return {"seconds": dt, "ms_per_step": 1e3 * dt / steps, "updates_per_s": updates / dt,
                "sweeps": [r["sweeps"] for r in reps[-1]], "outer": [r["outer"] for r in reps[-1]],
                "rel_res": [r["rel_res"] for r in reps[-1]], "stats": st}


def cpu_baseline(mesh, Q, om, bs, colour, gpu_sweeps):
    """The oracle as it stands, on one host core, on a bounded sample of the same
    workload: assembly of K, DILU factorisation of one harmonic system and two sweeps,
    timed separately; the step time is extrapolated to 4 systems x the GPU's sweep
    counts (assembly once, 4 factorisations, sum of sweeps)."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import assemble, solve
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        K = assemble.assemble(mesh, Q, eps=0.6, sigma=50.0)
        t_asm = time.perf_counter() - t0
        t0 = time.perf_counter()
        f = solve.factor(K, mesh.volume, mesh.zone, om[1], colour, "DILU")
        t_fac = time.perf_counter() - t0
        Ds = solve.system_diag(K, mesh.volume, mesh.zone, om[1])
        x = np.zeros_like(bs[1])
        n_sw = 2
        t0 = time.perf_counter()
        for _ in range(n_sw):
            r = bs[1] - solve.apply(K, Ds, x)
            x = x + solve.precondition(K, f, r)
        t_sw = (time.perf_counter() - t0) / n_sw
    t_step = t_asm + len(bs) * t_fac + sum(gpu_sweeps) * t_sw
    updates = mesh.n_cells * sum(gpu_sweeps)
    return {"value": updates / t_step, "unit": "cell-unknown updates/s", "cores": 1, "kind": "oracle",
            "sample": (f"oracle (NumPy FP64) on the same 200k-cell mesh: assemble {t_asm:.2f} s, DILU factor of one "
                       f"system {t_fac:.2f} s, {t_sw:.2f} s per sweep (mean of {n_sw}); step time extrapolated to "
                       f"{len(bs)} systems x GPU sweep counts {gpu_sweeps} = {t_step:.1f} s"),
            "extrapolated_step_s": t_step}


def learned_compare(mesh, Q, om, bs, storage, n_pairs, train_steps, batch, learn_every, reps=3, lr=1e-3, seed=0):
    """Learned preconditioner against the plain sweep on the same systems: training pairs
    from the plain solver (b = 0, random start, m DILU sweeps: the iterate is minus its
    error, its residual -K x), Adam on the GPU, then both solves to the 1e-8 drop, as
    Richardson sweeps and as FGMRES(10) with the plain and the learned preconditioner."""
    import numpy as np
    import torch
    from paper_2404_01407_amd import fnlh
    from paper_2404_01407_amd.synth import he_init
    ctx = fnlh.Context(mesh, storage=storage, outer="exact")
    ctx.assemble_jacobian(torch.from_numpy(Q).cuda(), eps=0.6, sigma=50.0)
    ctx.set_harmonics(om)
    S, N = len(bs), mesh.n_cells
    bd = [torch.from_numpy(b).cuda() for b in bs]

    def solve(kind):
        times, rep = [], None
        for _ in range(reps):
            xs = [torch.zeros_like(b) for b in bd]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, rep = ctx.relax(list(range(S)), xs, bd, kind=kind, max_sweeps=4000, rtol=RTOL, check_every=16,
                                use_graph=True, learn_every=learn_every)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            if st not in CONVERGED:
                raise RuntimeError(f"{kind} solve did not converge: {rep}")
        ms = 1e3 * float(np.median(times))
        return {"ms": round(ms, 3), "sweeps": [r["sweeps"] for r in rep], "outer": [r["outer"] for r in rep],
                "rel_res": [r["rel_res"] for r in rep], "learned_steps": [r["learned"] for r in rep],
                "rejected": [r["fallbacks"] for r in rep],
                "updates_per_s": round(N * sum(r["sweeps"] for r in rep) / (ms * 1e-3))}

    plain = solve("dilu")
    net = fnlh.Network(ctx)
    net.set_weights(he_init(seed))
    net.reserve_pairs(n_pairs)
    zero = torch.zeros(N, 6, dtype=torch.complex128, device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(1234 + seed)
    sweep_choices = [4, 8, 16, 32, 64, 128]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    k = 0
    while net.n_pairs() < n_pairs:
        m = sweep_choices[k % len(sweep_choices)]
        take = min(S, n_pairs - net.n_pairs())
        xs = [torch.randn(N, 6, dtype=torch.complex128, device="cuda", generator=gen) for _ in range(take)]
        ctx.relax(list(range(take)), xs, [zero] * take, kind="dilu", max_sweeps=m, rtol=0.0, check_every=16,
                  use_graph=True)
        for j in range(take):
            r = torch.empty_like(xs[j])
            ctx.residual(j, xs[j], zero, r)
            net.add_pairs([j], [r], [-xs[j]])
        k += 1
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    t0 = time.perf_counter()
    hist = net.train(train_steps, batch=batch, lr=lr, seed=seed + 1)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    learned = solve("learned")

    def fgmres(kind):
        # FGMRES(10), one DILU sweep per preconditioner application, after the learned
        # step for kind "learned" (the flexible method admits the nonlinear preconditioner)
        times, rep = [], None
        for _ in range(reps):
            xs = [torch.zeros_like(b) for b in bd]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, rep = ctx.gmres(list(range(S)), xs, bd, kind=kind, restart=10, max_iters=2000, rtol=RTOL,
                                use_graph=True)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            if st not in CONVERGED:
                raise RuntimeError(f"FGMRES {kind} did not converge: {rep}")
        return {"ms": round(1e3 * float(np.median(times)), 3), "iters": [r["iters"] for r in rep],
                "learned_steps": [r["learned"] for r in rep], "rel_res": [r["rel_res"] for r in rep]}

    fg = {"dilu": fgmres("dilu"), "learned": fgmres("learned")}
    fg["speedup_time"] = round(fg["dilu"]["ms"] / fg["learned"]["ms"], 3)
    fg["iter_ratio"] = round(sum(fg["dilu"]["iters"]) / max(sum(fg["learned"]["iters"]), 1), 3)
    q = max(1, len(hist) // 10)
    out = {"storage": storage, "learn_every": learn_every, "plain": plain, "learned": learned,
           "speedup_time": round(plain["ms"] / learned["ms"], 3),
           "sweep_ratio": round(sum(plain["sweeps"]) / max(sum(learned["sweeps"]), 1), 3), "fgmres": fg,
           "training": {"pairs": n_pairs, "pair_sweeps": sweep_choices, "steps": train_steps, "batch": batch,
                        "lr": lr, "generate_s": round(t_gen, 2), "train_s": round(t_train, 2),
                        "ms_per_sample": round(1e3 * t_train / max(train_steps * batch, 1), 3),
                        "loss_first": round(float(np.mean(hist[:q])), 4),
                        "loss_last": round(float(np.mean(hist[-q:])), 4)}}
    net.close()
    ctx.close()
    return out


def run_learned(args):
    mesh, Q, om, bs = build_inputs()
    print(f"[bench] learned: {mesh.n_cells} cells, {len(bs)} systems, {args.pairs} pairs, {args.train_steps} steps",
          file=sys.stderr, flush=True)
    res = learned_compare(mesh, Q, om, bs, args.storage, args.pairs, args.train_steps, args.batch, args.learn_every,
                          reps=max(args.steps, 1))
    print(f"[bench] plain {res['plain']['ms']} ms, learned {res['learned']['ms']} ms", file=sys.stderr, flush=True)
    out = {
        "metric": METRIC,
        "value": res["learned"]["updates_per_s"],
        "unit": "cell-unknown updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": 0,
        "ms_per_step": res["learned"]["ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16 network (f32 accumulate), " + args.storage + " blocks, f64 outer residual",
        "data": "synthetic",
        "config": {"workload": ("learned preconditioner: 200k-cell hex passage sector 80x50x50, mean + 3 harmonics; "
                                "network trained on the GPU on plain-solver residual/error pairs, then learned vs "
                                "plain DILU sweeps to a 1e-8 residual drop"),
                   "cells": mesh.n_cells, "systems": len(bs)},
        "time_to_1e-8_ms": {"plain": res["plain"]["ms"], "learned": res["learned"]["ms"]},
        "learned": res,
    }
    print(json.dumps(out), flush=True)


LARGEST_PROFILE = "k_rb_pass_update_f32_1920k_mean10h.md"


def calib_copy():
    """A plain elementwise kernel of known traffic for the counter calibration:
    torch.neg over 1 GiB (reads 1 GiB, writes 1 GiB), three times."""
    import torch
    xs = torch.ones(256 * 1024 * 1024, dtype=torch.float32, device="cuda")
    ys = torch.empty_like(xs)
    for _ in range(3):
        torch.neg(xs, out=ys)
    torch.cuda.synchronize()
    del xs, ys
    print("[bench] calibration: torch.neg over 1 GiB (read 1 GiB, write 1 GiB) x3", file=sys.stderr, flush=True)


def kernel_sources_sha():
    """Fingerprint of the sweep kernels' sources (comments and layout stripped): a
    counter summary taken with other code no longer describes the kernel this build
    launches."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in ("kernels.hip", "kernels.h", "device.h"):
        with open(os.path.join(ROOT, "paper_2404_01407_amd", "csrc", f)) as fh:
            code = fh.read()
        code = re.sub(r"/\*.*?\*/", " ", code, flags=re.S)
        code = re.sub(r"//[^\n]*", " ", code)
        h.update(" ".join(code.split()).encode())
    return h.hexdigest()[:16]


def traffic_from_profile(name):
    """HBM bytes per launch of the dominant kernel from the committed counter summary
    (its line 'traffic_bytes_per_launch <bytes> sources <sha16>', FETCH_SIZE and
    WRITE_SIZE scaled by the copy-kernel calibration); (None, why) when the summary is
    missing or was taken with other kernel sources."""
    import re
    try:
        with open(os.path.join(ROOT, "profiles", name)) as fh:
            text = fh.read()
    except OSError:
        return None, f"profiles/{name} missing"
    m = re.search(r"traffic_bytes_per_launch\s+(\d+)\s+sources\s+([0-9a-f]{16})", text)
    if not m:
        return None, f"no traffic line in profiles/{name}"
    if m.group(2) != kernel_sources_sha():
        return None, "kernel sources changed since the counter runs"
    return int(m.group(1)), f"profiles/{name}"


def precision_profile_name(storage, n_cells):
    return f"k_rb_pass_{storage}_{n_cells // 1000}k_mean3h.md"


def build_largest(shape):
    import numpy as np  # noqa: F401
    from paper_2404_01407_amd import synth
    mesh = synth.multi_row(*shape, n_blades=(36, 60, 48), seed=5)
    Q = synth.flow_state(mesh, 5)
    n_h = 10
    om = synth.omegas_multi_row(n_h, (36, 60, 48))
    bs = [synth.rhs(mesh.n_cells, s, real=(s == 0)) for s in range(n_h + 1)]
    return mesh, Q, om, bs


_POOL = {}


def _pool_worker(s):
    """One system's DILU factorisation and one sweep of the oracle in a forked worker
    (K, mesh and colouring inherited from the parent), on one thread."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import solve
    g = _POOL
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        f = solve.factor(g["K"], g["mesh"].volume, g["mesh"].zone, g["om"][s], g["colour"], "DILU")
        t_fac = time.perf_counter() - t0
        Ds = solve.system_diag(g["K"], g["mesh"].volume, g["mesh"].zone, g["om"][s])
        x = np.zeros_like(g["bs"][s])
        t0 = time.perf_counter()
        r = g["bs"][s] - solve.apply(g["K"], Ds, x)
        x = x + solve.precondition(g["K"], f, r)
        t_sw = time.perf_counter() - t0
    return t_fac, t_sw


def cpu_sample_largest(mesh, Q, om, bs, colour, pool_workers):
    """The oracle as it stands, timed on a bounded sample of the same workload before the
    GPU is touched: assembly of K, then (1) on one thread the DILU factorisation of one
    harmonic system and one sweep, (2) a process pool with one system per worker (the
    systems are decoupled), every system's factorisation and one sweep.  Step times are
    extrapolated to the GPU's sweep counts afterwards (cpu_baseline_from)."""
    import multiprocessing as mp
    from threadpoolctl import threadpool_limits
    from oracle import assemble
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        K = assemble.assemble(mesh, Q, eps=0.6, sigma=50.0)
        t_asm = time.perf_counter() - t0
    _POOL.update(K=K, mesh=mesh, om=om, bs=bs, colour=colour)
    t_fac1, t_sw1 = _pool_worker(1)
    S = len(bs)
    W = max(1, min(S, pool_workers))
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(W) as pool:
        res = pool.map(_pool_worker, range(S), chunksize=1)
    t_pool = time.perf_counter() - t0
    _POOL.clear()
    return {"t_asm": t_asm, "t_fac1": t_fac1, "t_sw1": t_sw1, "workers": W, "t_pool_wall": t_pool,
            "pool": res, "cpu_count": os.cpu_count()}


def cpu_baseline_from(sample, n_cells, gpu_sweeps, label):
    """Extrapolate the sampled oracle costs to the GPU's sweep counts: one thread
    (assembly + every factorisation + every sweep in turn) and the pool (assembly, then
    the systems spread over the workers, each factorisation and its sweeps)."""
    S = len(gpu_sweeps)
    t_single = sample["t_asm"] + S * sample["t_fac1"] + sum(gpu_sweeps) * sample["t_sw1"]
    W = sample["workers"]
    per_sys = [f + n * sw for (f, sw), n in zip(sample["pool"], gpu_sweeps)]
    loads = [0.0] * W
    for t in sorted(per_sys, reverse=True):  # longest first onto the least-loaded worker
        loads[loads.index(min(loads))] += t
    t_pool = sample["t_asm"] + max(loads)
    updates = n_cells * sum(gpu_sweeps)
    return {"value": updates / t_pool, "unit": "cell-system-sweep updates/s", "cores": W, "kind": "oracle",
            "sample": (f"oracle (NumPy FP64) on the {label}: assembly {sample['t_asm']:.1f} s (1 thread); "
                       f"pool of {W} processes (one thread each, os.cpu_count() = {sample['cpu_count']}): every "
                       f"system's DILU factorisation and one sweep, {sample['t_pool_wall']:.1f} s wall; step "
                       f"extrapolated to the GPU sweep counts = {t_pool:.1f} s"),
            "extrapolated_step_s": round(t_pool, 2),
            "single_thread": {"value": updates / t_single, "cores": 1,
                              "factor_s": round(sample["t_fac1"], 2), "sweep_s": round(sample["t_sw1"], 2),
                              "extrapolated_step_s": round(t_single, 1)},
            "cpu_count": sample["cpu_count"]}


def train_heldout(storage, meshes_seeds, starts, snapshots, every, rounds, steps_per_round, batch, lr, seed=0):
    """The learned preconditioner's training protocol: pairs from the plain solver on
    training meshes (200k-cell passages, one seed each, mean + 3 harmonics), generated in
    the library (random starts, a snapshot every `every` DILU sweeps), then Adam on the
    GPU, a round of steps on each mesh in turn (the state moves device to device).
    Returns (checkpoint path, report)."""
    import tempfile
    import numpy as np
    import torch
    from paper_2404_01407_amd import fnlh, synth
    ctxs, nets = [], []
    t0 = time.perf_counter()
    for sd in meshes_seeds:
        m = synth.passage_block(*SHAPE, 36, seed=sd)
        c = fnlh.Context(m, storage=storage, outer="exact")
        c.assemble_jacobian(torch.from_numpy(synth.flow_state(m, sd)).cuda(), eps=0.6, sigma=50.0)
        c.set_harmonics(synth.omegas_single_zone(N_HARM, 36))
        n = fnlh.Network(c)
        n.reserve_pairs((N_HARM + 1) * starts * snapshots)
        ctxs.append(c)
        nets.append(n)
    t_setup = time.perf_counter() - t0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k, n in enumerate(nets):
        n.generate(list(range(N_HARM + 1)), starts, snapshots, every, seed=1000 + k)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    nets[0].set_weights(synth.he_init(seed))
    hist = []
    t0 = time.perf_counter()
    prev = nets[0]
    for r in range(rounds):
        for k, n in enumerate(nets):
            if n is not prev:
                n.copy_state_from(prev)
            hist.append(n.train(steps_per_round, batch=batch, lr=lr, seed=seed + 17 * r + k))
            prev = n
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    path = os.path.join(tempfile.mkdtemp(prefix="fnlh_"), "net.fnlhnn")
    prev.save(path)
    h = np.concatenate(hist)
    q = max(1, len(h) // 10)
    pairs = sum(n.n_pairs() for n in nets)
    for n, c in zip(nets, ctxs):
        n.close()
        c.close()
    return path, {"train_meshes": [f"passage_block{SHAPE} seed {s}" for s in meshes_seeds], "pairs": pairs,
                  "snapshot_every": every, "snapshots_per_start": snapshots, "adam_steps": len(h), "batch": batch,
                  "lr": lr, "setup_s": round(t_setup, 2), "generate_s": round(t_gen, 2),
                  "train_s": round(t_train, 2), "ms_per_sample": round(1e3 * t_train / max(len(h) * batch, 1), 3),
                  "loss_first": round(float(np.mean(h[:q])), 4), "loss_last": round(float(np.mean(h[-q:])), 4)}


def time_solve(ctx, bd, kind, reps, learn_every=32, max_sweeps=6000):
    """Median wall time of a whole solve to the 1e-8 drop (graph replay) and its report."""
    import numpy as np
    import torch
    times, rep, st = [], None, 0
    S = len(bd)
    for _ in range(reps):
        xs = [torch.zeros_like(b) for b in bd]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, rep = ctx.relax(list(range(S)), xs, bd, kind=kind, max_sweeps=max_sweeps, rtol=RTOL, check_every=16,
                            use_graph=True, learn_every=learn_every)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        if st not in CONVERGED:
            raise RuntimeError(f"{kind} solve did not converge: {rep}")
    return {"ms": round(1e3 * float(np.median(times)), 3), "status": st, "sweeps": [r["sweeps"] for r in rep],
            "outer": [r["outer"] for r in rep], "learned_steps": [r["learned"] for r in rep],
            "rejected": [r["fallbacks"] for r in rep], "fell_back": sum(r["status"] == 3 for r in rep),
            "rel_res": [r["rel_res"] for r in rep]}


def learned_eval(ctx, bd, ckpt, reps, learn_every, plain=None):
    """Plain DILU against learned + DILU (+ FP64 defect correction in reduced precision) on
    ctx's systems with the trained network loaded from ckpt."""
    from paper_2404_01407_amd import fnlh
    if plain is None:
        plain = time_solve(ctx, bd, "dilu", reps)
    net = fnlh.Network(ctx)
    net.load(ckpt)
    learned = time_solve(ctx, bd, "learned", reps, learn_every)
    net.close()
    return {"plain": plain, "learned": learned, "speedup_time": round(plain["ms"] / learned["ms"], 3),
            "sweep_ratio": round(sum(plain["sweeps"]) / max(sum(learned["sweeps"]), 1), 3)}


def heldout_eval(storage, ckpt, reps, learn_every, seed=14):
    """The held-out test of the learned preconditioner: a 200k-cell passage of a seed no
    pair came from, mean + 3 harmonics."""
    import torch
    from paper_2404_01407_amd import fnlh, synth
    m = synth.passage_block(*SHAPE, 36, seed=seed)
    c = fnlh.Context(m, storage=storage, outer="exact")
    c.assemble_jacobian(torch.from_numpy(synth.flow_state(m, seed)).cuda(), eps=0.6, sigma=50.0)
    c.set_harmonics(synth.omegas_single_zone(N_HARM, 36))
    bd = [torch.from_numpy(synth.rhs(m.n_cells, s, real=(s == 0))).cuda() for s in range(N_HARM + 1)]
    res = learned_eval(c, bd, ckpt, reps, learn_every)
    res["mesh"] = f"passage_block{SHAPE} seed {seed} (held out)"
    c.close()
    return res


def precision_summary(args):
    """The 200k-cell precision configuration as a sub-field: time to 1e-8 and the error of
    each block precision's solution against the FP64 one (FP64 is held to the oracle by
    the parity tests)."""
    import torch
    mesh, Q, om, bs = build_inputs()
    sols, out = {}, {}
    for s in ("f64", "f32", "bf16"):
        r = Runner(mesh, Q, om, bs, s, check_every=16, use_graph=True)
        m = r.timed(3, 1)
        sols[s] = [x.clone() for x in r.xd]
        out[s] = {"ms_per_step": round(m["ms_per_step"], 3), "updates_per_s": round(m["updates_per_s"]),
                  "sweeps": m["sweeps"], "outer": m["outer"]}
        r.ctx.close()
    for s in ("f32", "bf16"):
        out[s]["err_vs_f64"] = [float(torch.linalg.norm(a - b) / torch.linalg.norm(b))
                                for a, b in zip(sols[s], sols["f64"])]
    return {"workload": "200k-cell passage 80x50x50, mean + 3 harmonics, DILU to 1e-8", "by_storage": out}


def run_largest(args):
    """The headline: three-row sector (rotor-stator-rotor, 3 x 100x64x100 = 1.92M cells
    plus the pitch-overlap interface couplings, greedy colouring: two large colours and a
    remainder of interface rows), mean + 10 harmonics at mixed per-row frequencies, one
    shared Jacobian in FP32 with the FP64 defect correction, DILU sweeps (two-colour
    passes plus remainder passes) to a 1e-8 residual drop.  One step = assemble K, set the
    harmonics, factor the 11 systems, sweep all of them to 1e-8 with the FP64 outer
    residual.  The last timed step also times every sweep-pass launch with HIP events."""
    import numpy as np
    import torch
    from paper_2404_01407_amd import fnlh
    t0 = time.perf_counter()
    mesh, Q, om, bs = build_largest(args.largest_shape)
    S = len(bs)
    print(f"[bench] largest: {mesh.n_cells} cells, {mesh.n_edges} faces, {S} systems, inputs "
          f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    colour, _, n_col = fnlh.order_mesh(mesh)
    sample = None
    if not args.no_cpu_baseline:
        # the oracle sample runs before the GPU is initialised (its process pool forks)
        print("[bench] timing the CPU oracle sample", file=sys.stderr, flush=True)
        sample = cpu_sample_largest(mesh, Q, om, bs, colour, min(16, os.cpu_count() or 1))
        print(f"[bench] oracle sample: assembly {sample['t_asm']:.1f} s, factor {sample['t_fac1']:.1f} s, sweep "
              f"{sample['t_sw1']:.1f} s, pool of {sample['workers']} {sample['t_pool_wall']:.1f} s", file=sys.stderr,
              flush=True)
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.calib_copy:
        calib_copy()
    t0 = time.perf_counter()
    ctx = fnlh.Context(mesh, storage=args.storage, outer="exact")
    ingest_ms = 1e3 * (time.perf_counter() - t0)
    ctx.tune(hybrid=args.hybrid)
    Qd = torch.from_numpy(Q).cuda()
    bd = [torch.from_numpy(b).cuda() for b in bs]
    mem = {}
    for k in (1, 3, 6, S):
        ctx.assemble_jacobian(Qd, eps=0.6, sigma=50.0)
        ctx.set_harmonics(om[:k])
        xs = [torch.zeros_like(b) for b in bd[:k]]
        ctx.relax(list(range(k)), xs, bd[:k], kind="dilu", max_sweeps=2, rtol=0.0, check_every=2)
        mem[k] = ctx.memory()
        del xs
    print(f"[bench] largest: memory by system count {mem}", file=sys.stderr, flush=True)
    xd = [torch.zeros_like(b) for b in bd]

    def step():
        for x in xd:
            x.zero_()
        ctx.assemble_jacobian(Qd, eps=0.6, sigma=50.0)
        ctx.set_harmonics(om)
        st, rep = ctx.relax(list(range(S)), xd, bd, kind="dilu", max_sweeps=6000, rtol=RTOL, check_every=16,
                            use_graph=not args.no_graph)
        if st not in CONVERGED:
            raise RuntimeError(f"largest: solve did not converge: {rep}")
        return rep

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = []
    for i in range(args.steps):
        if i == args.steps - 1 and not args.no_stats:
            ctx.stats_enable(True, period=1)  # events around every sweep-pass launch of the last step
        reps.append(step())
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    stats = ctx.stats()
    ctx.stats_enable(False)
    rep = reps[-1]
    sweeps = [r["sweeps"] for r in rep]
    updates_per_step = [mesh.n_cells * sum(r["sweeps"] for r in rp) for rp in reps]
    print(f"[bench] largest: {1e3 * dt:.1f} ms/step, sweeps {sweeps}", file=sys.stderr, flush=True)
    kernels = {}
    for name, k in stats.items():
        if k["launches"]:
            ms = k["total_ms"] / k["launches"]
            kernels[name] = {"launches": k["launches"], "avg_launch_us": round(1e3 * ms, 2),
                             "alg_bytes_per_launch": round(k["alg_bytes"] / k["launches"]),
                             "achieved_GBs": round(k["alg_bytes"] / k["launches"] / (ms * 1e-3) / 1e9, 1)}
    sweep_kinds = [n for n in ("sweep_update", "sweep_set", "fwd", "fwd_last", "bwd", "remainder") if n in kernels]
    tot_ms = sum(stats[n]["total_ms"] for n in sweep_kinds)
    tot_b = sum(stats[n]["alg_bytes"] for n in sweep_kinds)
    dom = max(sweep_kinds, key=lambda n: stats[n]["total_ms"]) if sweep_kinds else None
    roofline = None
    if dom:
        kd = kernels[dom]
        names = {"sweep_update": "k_rb_pass<f32, update> (second-colour update pass)",
                 "sweep_set": "k_rb_pass<f32, set> (first-colour pass)", "fwd": "k_fwd<f32> (general forward)",
                 "bwd": "k_bwd<f32> (general backward)"}
        traffic, src = traffic_from_profile(LARGEST_PROFILE) if dom == "sweep_update" else (None, "no counter run")
        roofline = {"bound": "hbm", "achieved": kd["achieved_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(kd["achieved_GBs"] / HBM_PEAK_GBS, 4), "traffic": traffic,
                    "traffic_source": src, "kernel": names.get(dom, dom), "avg_launch_us": kd["avg_launch_us"],
                    "alg_bytes_per_launch": kd["alg_bytes_per_launch"], "launches": kd["launches"],
                    "all_sweep_kernels_GBs": round(tot_b / (tot_ms * 1e-3) / 1e9, 1) if tot_ms else None,
                    "all_sweep_kernels_frac": round(tot_b / (tot_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if tot_ms else None}
    learned = ckpt = None
    if not args.no_learned:
        print("[bench] learned: training on held-out-protocol pairs (seeds 10-13)", file=sys.stderr, flush=True)
        ckpt, training = train_heldout(args.storage, [10, 11, 12, 13], args.learn_starts, 8, 4, args.learn_rounds,
                                       8, 8, 1e-3)
        on5 = learned_eval(ctx, bd, ckpt, 1, args.learn_every, plain=time_solve(ctx, bd, "dilu", 1))
        print(f"[bench] learned on the sector: plain {on5['plain']['ms']} ms, learned {on5['learned']['ms']} ms",
              file=sys.stderr, flush=True)
        held = heldout_eval(args.storage, ckpt, 3, args.learn_every)
        print(f"[bench] learned on held-out seed 14: plain {held['plain']['ms']} ms, learned "
              f"{held['learned']['ms']} ms", file=sys.stderr, flush=True)
        learned = {"training": training, "on_this_workload": on5, "held_out_200k": held,
                   "learn_every": args.learn_every}
    colours = ctx.ordering()[1]
    ctx.close()
    precision = None
    if not args.no_modes:
        precision = precision_summary(args)
    batch = None
    if not args.no_batch:
        print("[bench] batching: 64 instances", file=sys.stderr, flush=True)
        batch = batch_measure(args, ckpt=ckpt if learned else None, steps=2, warmup=1,
                              training=learned["training"] if learned else None)
    cpu = cpu_baseline_from(sample, mesh.n_cells, sweeps, "same 1.92M-cell sector") if sample else None
    out = {
        "metric": METRIC,
        "value": round(sum(updates_per_step) / (dt * args.steps)),
        "unit": "cell-system-sweep updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * dt, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": _dtype_of(args.storage),
        "data": "synthetic",
        "config": {"workload": ("three-row sector rotor-stator-rotor 3 x 100x64x100 (36/60/48 blades, pitch-overlap "
                                "interfaces), mean + 10 harmonics at mixed per-row frequencies, one shared FP32 "
                                "Jacobian, DILU (two-colour + remainder passes) with FP64 defect correction to a "
                                "1e-8 residual drop"),
                   "cells": mesh.n_cells, "faces": mesh.n_edges, "systems": S, "colours": colours,
                   "storage": args.storage, "eps": 0.6, "sigma": 50.0},
        "time_to_1e-8_ms": round(1e3 * dt, 3),
        "sweeps": sweeps,
        "outer": [r["outer"] for r in rep],
        "rel_res": [r["rel_res"] for r in rep],
        "roofline": roofline,
        "cpu_baseline": cpu,
        "sweep_kernels": kernels,
        "memory_bytes_by_systems": {str(k): v for k, v in mem.items()},
        "learned": learned,
        "precision_200k": precision,
        "batching_8M": batch,
        "ingest_ms": round(ingest_ms, 1),
    }
    print(json.dumps(out), flush=True)


def run_phase(args):
    """Phase-lagged periodic boundaries: a 200k-cell linear-cascade passage (80 x 50 x 50,
    pitchwise sides joined by periodic edges), mean + 3 harmonics whose inter-blade phase
    angles follow from 60 upstream vanes against 36 blades (sigma_l = 2 pi l 60 / 36),
    FP32 blocks, DILU to 1e-8; the same solves without the phases for comparison."""
    import numpy as np
    import torch
    from paper_2404_01407_amd import fnlh, synth
    mesh = synth.cascade_block(80, 50, 50, 36, seed=2)
    Q = synth.flow_state(mesh, 2)
    om = synth.omegas_single_zone(N_HARM, 36)
    sigma = np.array([2.0 * np.pi * l * 60.0 / 36.0 for l in range(N_HARM + 1)])
    bs = [synth.rhs(mesh.n_cells, s, real=(s == 0)) for s in range(N_HARM + 1)]
    out = {}
    for phased in (True, False):
        r = Runner(mesh, Q, om, bs, args.storage, check_every=args.check_every, use_graph=not args.no_graph)
        if phased:
            # the step sets the harmonics, which resets the phases: apply them after it
            def step(ctx=r.ctx):
                for x in r.xd:
                    x.zero_()
                ctx.assemble_jacobian(r.Qd, eps=0.6, sigma=50.0)
                ctx.set_harmonics(om)
                ctx.set_phase_lag(mesh.edge_phase, sigma)
                st, rep = ctx.relax(list(range(r.S)), r.xd, r.bd, kind="dilu", max_sweeps=4000, rtol=RTOL,
                                    check_every=r.check_every, use_graph=r.use_graph)
                if st not in CONVERGED:
                    raise RuntimeError(f"phased solve did not converge: {rep}")
                return rep
            r.step = step
        res = r.timed(args.steps, args.warmup, stats=True)
        st = res["stats"]
        u = st["sweep_update"]
        au = u["total_ms"] / max(u["launches"], 1)
        out["phased" if phased else "no_phase"] = {
            "ms_per_step": round(res["ms_per_step"], 3), "updates_per_s": round(res["updates_per_s"]),
            "sweeps": res["sweeps"], "rel_res": res["rel_res"],
            "update_pass_us": round(1e3 * au, 2),
            "update_pass_GBs": round(u["alg_bytes"] / max(u["launches"], 1) / (au * 1e-3) / 1e9, 1) if au else 0.0}
        colours = r.ctx.ordering()[1]
        r.ctx.close()
        print(f"[bench] phase ({'on' if phased else 'off'}): {res['ms_per_step']:.2f} ms/step, sweeps {res['sweeps']}",
              file=sys.stderr, flush=True)
    ph = out["phased"]
    res = {
        "metric": METRIC, "value": ph["updates_per_s"], "unit": "cell-unknown updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ph["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"f64": "f64", "f32": "f32 blocks, f32 sweep, f64 outer residual",
                  "bf16": "bf16 blocks, f32 sweep, f64 outer residual"}[args.storage],
        "data": "synthetic",
        "config": {"workload": ("200k-cell linear-cascade passage 80x50x50 with phase-lagged periodic sides, mean + 3 "
                                "harmonics, inter-blade phase angles 2 pi l 60/36, DILU to a 1e-8 residual drop"),
                   "cells": mesh.n_cells, "faces": mesh.n_edges, "periodic_faces": int(np.count_nonzero(mesh.edge_phase)),
                   "colours": colours, "storage": args.storage},
        "time_to_1e-8_ms": ph["ms_per_step"], "phase": out,
    }
    print(json.dumps(res), flush=True)


def _dtype_of(storage):
    return {"f64": "f64 blocks and factor inverses, f64 sweep",
            "f32": "f32 blocks, f16 factor inverses (power-of-two row scale), f32 sweep, f64 outer residual",
            "bf16": "bf16 blocks, f16 factor inverses (power-of-two row scale), f32 sweep, f64 outer residual"}[storage]


def run_krylov(args):
    """Restarted flexible GMRES against the plain Richardson iteration with the same DILU
    preconditioner: the 200k-cell passage, mean + 3 harmonics, time to a 1e-8 residual drop
    (assembly, harmonics and factorisation included in both)."""
    import torch
    mesh, Q, om, bs = build_inputs()
    r = Runner(mesh, Q, om, bs, args.storage, check_every=args.check_every, use_graph=not args.no_graph)
    last = {}

    def gmres_step(ctx=r.ctx):
        for x in r.xd:
            x.zero_()
        ctx.assemble_jacobian(r.Qd, eps=0.6, sigma=50.0)
        ctx.set_harmonics(om)
        st, rep = ctx.gmres(list(range(r.S)), r.xd, r.bd, kind="dilu", restart=args.restart, max_iters=2000,
                            rtol=RTOL, inner_sweeps=args.inner_sweeps)
        if st not in CONVERGED:
            raise RuntimeError(f"gmres did not converge: {rep}")
        last["rep"] = rep
        return [{"sweeps": q["iters"] * args.inner_sweeps, "outer": q["restarts"], "rel_res": q["rel_res"]}
                for q in rep]

    plain = r.timed(args.steps, args.warmup)
    print(f"[bench] krylov: Richardson {plain['ms_per_step']:.2f} ms/step, sweeps {plain['sweeps']}", file=sys.stderr,
          flush=True)
    r.step = gmres_step
    gm = r.timed(args.steps, args.warmup)
    print(f"[bench] krylov: FGMRES({args.restart}) {gm['ms_per_step']:.2f} ms/step, iterations "
          f"{[q['iters'] for q in last['rep']]}", file=sys.stderr, flush=True)
    colours = r.ctx.ordering()[1]
    r.ctx.close()
    torch.cuda.synchronize()
    res = {
        "metric": METRIC, "value": round(gm["updates_per_s"]), "unit": "cell-unknown updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(gm["ms_per_step"], 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": _dtype_of(args.storage),
        "data": "synthetic",
        "config": {"workload": (f"200k-cell passage 80x50x50, mean + 3 harmonics, FGMRES({args.restart}) with "
                                f"{args.inner_sweeps} DILU sweep(s) per preconditioner application vs DILU "
                                "Richardson, to a 1e-8 residual drop"),
                   "cells": mesh.n_cells, "colours": colours, "storage": args.storage},
        "fgmres": {"ms_per_step": round(gm["ms_per_step"], 3), "iterations": [q["iters"] for q in last["rep"]],
                   "restarts": [q["restarts"] for q in last["rep"]], "rel_res": gm["rel_res"]},
        "richardson": {"ms_per_step": round(plain["ms_per_step"], 3), "sweeps": plain["sweeps"],
                       "rel_res": plain["rel_res"]},
        "fgmres_speedup_vs_richardson": round(plain["ms_per_step"] / gm["ms_per_step"], 3),
    }
    print(json.dumps(res), flush=True)


def run_rk(args):
    """The RK(5,3) pseudo-time driver around the solve: the 200k-cell passage, implicit
    scheme (eps 0.6, sigma 50), paper-mode stage solves (DILU, 1e-2, at most 10 sweeps);
    per pseudo-time step the mean flow (K re-assembled, five stage solves with the Rusanov
    residual) and three harmonics (five stage solves each with the linearised residual)."""
    import numpy as np
    import torch
    from paper_2404_01407_amd import fnlh, synth
    mesh, Q, om, bs = build_inputs()
    ctx = fnlh.Context(mesh, storage=args.storage, outer="exact")
    state = torch.from_numpy(Q).cuda()
    ctx.assemble_jacobian(state)
    ctx.set_harmonics(om)
    rng = np.random.default_rng(3)
    fh = [torch.from_numpy(rng.standard_normal((mesh.n_cells, 6)) + 1j * rng.standard_normal((mesh.n_cells, 6))).cuda()
          for _ in range(N_HARM)]
    qh = [torch.zeros_like(f) for f in fh]
    hist_m, hist_h = [], [[] for _ in range(N_HARM)]

    def step():
        _, hm = ctx.rk_mean(0, state, 1, eps=0.6, sigma=50.0, max_sweeps=10, rtol=1e-2)
        hist_m.extend(hm.tolist())
        for l in range(N_HARM):
            _, hh = ctx.rk_harmonic(l + 1, qh[l], fh[l], 1, max_sweeps=10, rtol=1e-2)
            hist_h[l].extend(hh.tolist())

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.close()
    ms = 1e3 * dt / args.steps
    print(f"[bench] rk: {ms:.2f} ms per pseudo-time step (mean + {N_HARM} harmonics)", file=sys.stderr, flush=True)
    stage_solves = 5 * (1 + N_HARM)
    res = {
        "metric": "pseudo-time steps/s", "value": round(1e3 / ms, 3), "unit": "pseudo-time steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": _dtype_of(args.storage), "data": "synthetic",
        "config": {"workload": ("200k-cell passage 80x50x50, RK(5,3) pseudo-time steps of the mean flow and 3 "
                                "harmonics, implicit scheme, paper-mode DILU stage solves (1e-2, at most 10 sweeps)"),
                   "cells": mesh.n_cells, "storage": args.storage},
        "stage_solves_per_step": stage_solves,
        "mean_residual_first_last": [hist_m[0], hist_m[-1]],
        "harmonic_residual_first_last": [[h[0], h[-1]] for h in hist_h],
        # the paper's harmonic residual monitor: R_z = sqrt(mean over the harmonics of the
        # squared RMS of each harmonic's residual), RMS over the 6N complex entries
        "R_z_per_step": [float(np.sqrt(np.mean([(h[k] ** 2) / (6 * mesh.n_cells) for h in hist_h])))
                         for k in range(len(hist_h[0]))],
        "mean_rms_per_step": [float(v / np.sqrt(6 * mesh.n_cells)) for v in hist_m],
    }
    print(json.dumps(res), flush=True)


def run_partition_ilu(args):
    """Partition-local ILU(0) (section "Parallel Implementation": each partition solves
    its own block of the LHS, the couplings to other partitions ignored) against the
    colour-ordered DILU on the same dropped matrix and on the whole matrix: one harmonic
    system at the BPF on the 200k-cell passage, preconditioned Richardson to a 1e-6
    residual drop from zero; sweeps, time per sweep and per solve by partition size.  The
    natural order is the mesh's cell numbering: the structured (axial, pitch, radial)
    numbering of the generator, and a random renumbering for comparison."""
    import numpy as np
    import torch
    from paper_2404_01407_amd import fnlh, synth
    if args.calib_copy:
        calib_copy()
    shape = tuple(args.shape)
    out = []
    for numbering in args.part_numbering:
        mesh = synth.passage_block(*shape, 36, seed=2, permute=(numbering == "random"))
        Q = synth.flow_state(mesh, 2)
        ns = args.pilu_systems
        om = synth.omegas_single_zone(max(ns, 1), 36)
        sysl = list(range(1, ns + 1))
        bl = [torch.from_numpy(synth.rhs(mesh.n_cells, s)).cuda() for s in sysl]
        Qd = torch.from_numpy(Q).cuda()
        print(f"[bench] partition_ilu: {numbering} numbering, {mesh.n_cells} cells", file=sys.stderr, flush=True)
        for size in [mesh.n_cells] + [int(v) for v in args.pilu_sizes]:
            whole = size >= mesh.n_cells
            part = None if whole else synth.rcb_partition(mesh, size)
            ctx = fnlh.Context(mesh, storage=args.storage, outer="exact")
            if args.pilu_unit is not None or args.pilu_threads is not None:
                ctx.tune(pilu_unit=args.pilu_unit, pilu_threads=args.pilu_threads)
            if part is not None:
                ctx.set_partitions(part)
            ctx.assemble_jacobian(Qd, eps=0.6, sigma=50.0)
            ctx.set_harmonics(om)
            kinds = ["dilu"] if whole else ["dilu", "pilu"]
            if whole and numbering != args.part_numbering[0]:
                kinds = []  # the colour ordering does not depend on the numbering
            for kind in kinds:
                xl = [torch.zeros_like(b) for b in bl]
                best = None
                for rep_i in range(3):  # the first solve factors, builds tables and captures graphs
                    for x in xl:
                        x.zero_()
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    st, rep = ctx.relax(sysl, xl, bl, kind=kind, max_sweeps=args.pilu_max_sweeps, rtol=1e-6,
                                        check_every=16, use_graph=True)
                    torch.cuda.synchronize()
                    dt = 1e3 * (time.perf_counter() - t0)
                    r = max(rep, key=lambda d: d["sweeps"])
                    if rep_i and (best is None or dt < best[0]):
                        best = (dt, r)
                dt, r = best
                ctx.stats_enable(True)
                for x in xl:
                    x.zero_()
                ctx.relax(sysl, xl, bl, kind=kind, max_sweeps=32, rtol=0.0, check_every=16)
                torch.cuda.synchronize()
                ks = ctx.stats()
                ctx.stats_enable(False)
                launched = {k: v for k, v in ks.items() if v["launches"]}
                kern_ms = sum(v["total_ms"] for v in launched.values())
                kern_bytes = sum(v["alg_bytes"] for v in launched.values())
                rec = {"numbering": numbering, "kind": kind,
                       "cells_per_part": int(round(mesh.n_cells / (1 if part is None else int(part.max()) + 1))),
                       "parts": 1 if part is None else int(part.max()) + 1,
                       "max_part": mesh.n_cells if part is None else int(np.bincount(part).max()),
                       "status": int(r["status"]), "sweeps": int(r["sweeps"]), "rel_res": r["rel_res"],
                       "solve_ms": round(dt, 3), "factor_ms": round(r["t_factor_ms"], 3),
                       "sweep_ms": round(kern_ms / 32, 4),
                       "sweep_alg_GBs": round(kern_bytes / kern_ms / 1e6, 1) if kern_ms > 0 else None}
                print(f"[bench] partition_ilu: {rec}", file=sys.stderr, flush=True)
                out.append(rec)
            ctx.close()
    base = out[0]
    res = {
        "metric": "time to a 1e-6 residual drop by partition size", "value": base["solve_ms"], "unit": "ms",
        "n_gpus": 1, "steps": 1, "warmup": 2, "ms_per_step": base["solve_ms"], "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": _dtype_of(args.storage), "data": "synthetic",
        "config": {"workload": (f"{shape[0]}x{shape[1]}x{shape[2]} passage, {args.pilu_systems} harmonic(s) from the "
                                "BPF up, Richardson "
                                "to 1e-6 from zero: colour-ordered DILU on the whole and on the "
                                "partition-dropped matrix, partition-local natural-order ILU(0) (one "
                                "workgroup per partition, y in LDS) by partition size"),
                   "cells": int(np.prod(shape)), "storage": args.storage},
        "runs": out,
    }
    print(json.dumps(res), flush=True)


def run_partition(args):
    """The paper's parallel scheme on one GPU: the couplings between partitions of a
    recursive-bisection decomposition are dropped from K (each partition solves its own
    sub-system) and the RK(5,3) iteration of a harmonic (BPF, implicit, paper-mode DILU
    stage solves) is run to a 1e-6 residual drop; pseudo-time steps needed and time per
    partition size and CFL number on the 200k-cell passage, with the explicit scheme
    (K = P, CFL 1) as the single-cell limit."""
    import numpy as np
    import torch
    from paper_2404_01407_amd import fnlh, synth
    mesh, Q, om, bs = build_inputs()
    omh = om[:2]
    rng = np.random.default_rng(5)
    fh = torch.from_numpy(rng.standard_normal((mesh.n_cells, 6)) + 1j * rng.standard_normal((mesh.n_cells, 6))).cuda()
    Qd = torch.from_numpy(Q).cuda()

    def run(size, sigma, scheme, kind="dilu"):
        part = synth.rcb_partition(mesh, size)
        ctx = fnlh.Context(mesh, storage=args.storage, outer="exact")
        ctx.set_partitions(part)
        ctx.assemble_jacobian(Qd, eps=0.6, sigma=sigma, scheme=scheme)
        ctx.set_harmonics(omh)
        qh = torch.zeros_like(fh)
        hist = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        status = "not converged"
        while len(hist) < args.max_steps:
            _, h = ctx.rk_harmonic(1, qh, fh, 10, kind=kind, max_sweeps=10, rtol=1e-2)
            for r in h:
                hist.append(float(r))
                if r <= 1e-6 * hist[0]:
                    status = "converged"
                    break
                if not np.isfinite(r) or r > 1e3 * hist[0]:
                    status = "diverged"
                    break
            if status != "not converged":
                break
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ctx.close()
        rec = {"scheme": scheme, "kind": kind, "cfl": sigma,
               "cells_per_part": int(round(mesh.n_cells / (int(part.max()) + 1))),
               "parts": int(part.max()) + 1, "status": status, "steps": len(hist), "seconds": round(dt, 3),
               "final_drop": hist[-1] / hist[0]}
        print(f"[bench] partition: {rec}", file=sys.stderr, flush=True)
        return rec

    out = []
    for sigma in args.part_cfl:
        for size in [mesh.n_cells] + [int(v) for v in args.part_sizes]:
            out.append(run(size, float(sigma), "implicit"))
            # the partition-local ILU(0) stage solves where a partition fits in a workgroup
            if "pilu" in args.part_kinds and size < mesh.n_cells and \
                    np.bincount(synth.rcb_partition(mesh, size)).max() * (96 if args.storage == "f64" else 48) <= 162816:
                out.append(run(size, float(sigma), "implicit", "pilu"))
    out.append(run(mesh.n_cells, 1.0, "explicit"))
    base = out[0]
    res = {
        "metric": "pseudo-time steps to a 1e-6 residual drop", "value": base["steps"],
        "unit": "pseudo-time steps", "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": round(1e3 * base["seconds"], 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": _dtype_of(args.storage),
        "data": "synthetic",
        "config": {"workload": ("200k-cell passage 80x50x50, harmonic at the BPF, RK(5,3) implicit (eps 0.6) with "
                                "paper-mode DILU stage solves, couplings between recursive-bisection partitions "
                                "dropped from K; the explicit scheme (CFL 1) as the limit"),
                   "cells": mesh.n_cells, "storage": args.storage},
        "runs": out,
    }
    print(json.dumps(res), flush=True)


def batch_measure(args, ckpt=None, steps=None, warmup=1, training=None):
    """Batching workload: 64 independent blade-row instances, seeded log-uniform sizes in
    [20k, 300k] cells (~8M total), passage shapes (2n', n', n'), blade counts U{20..80},
    1-8 harmonics each (mean + harmonics, omega_l = l x BPF).  One step = relax every
    system of every instance to 1e-8 (FP32 blocks, FP64 outer residual), x0 = 0.
    Batched: one launch per colour phase and system-count group over the instances below
    the size threshold the batch autotuner picks, graph-replayed; baseline: the same
    solves issued instance by instance (graph-replayed as well).  The instance contexts
    are autotuned first (one per system count, whole-solve time).  With ckpt, the learned
    preconditioner (one trained state loaded into every instance's network) is timed in
    the batched form too."""
    import numpy as np
    import torch
    from paper_2404_01407_amd import fnlh, synth
    steps = args.steps if steps is None else steps
    specs = synth.batch_instances(args.instances, args.total_cells, seed=3)
    t0 = time.perf_counter()
    ctxs, systems, bd, xd, cells = [], [], [], [], 0
    for q, sp in enumerate(specs):
        m = synth.passage_block(*sp["shape"], sp["n_blades"], seed=sp["seed"])
        Q = synth.flow_state(m, sp["seed"])
        c = fnlh.Context(m, storage=args.storage)
        c.assemble_jacobian(torch.from_numpy(Q).cuda())
        nh = sp["n_harmonics"]
        c.set_harmonics(synth.omegas_single_zone(nh, sp["n_blades"]))
        ctxs.append(c)
        systems.append(list(range(nh + 1)))
        g = torch.Generator(device="cuda").manual_seed(1000 + q)
        row = []
        for s_ in range(nh + 1):
            re = torch.randn((m.n_cells, 6), generator=g, device="cuda", dtype=torch.float64)
            im = torch.zeros_like(re) if s_ == 0 else torch.randn((m.n_cells, 6), generator=g, device="cuda",
                                                                 dtype=torch.float64)
            row.append(torch.complex(re, im).contiguous())
        bd.append(row)
        xd.append([torch.zeros_like(b) for b in row])
        cells += m.n_cells
        del m, Q
        if q % 16 == 15:
            print(f"[bench] batch setup: {q + 1}/{len(specs)} instances, {cells} cells", file=sys.stderr, flush=True)
    setup_s = time.perf_counter() - t0
    n_sys_total = sum(len(sy) for sy in systems)
    print(f"[bench] batch: {len(ctxs)} instances, {cells} cells, {n_sys_total} systems, setup {setup_s:.1f} s",
          file=sys.stderr, flush=True)
    # autotune one representative per system count (whole solves to 1e-8), share the choice
    t0 = time.perf_counter()
    tuned = {}
    for c, sy in zip(ctxs, systems):
        k = len(sy)
        if k not in tuned:
            tuned[k] = c.autotune(k, rtol=RTOL)
        c.tune(tuned[k]["sys_per_lane"], tuned[k]["lanes_per_row"], wave_groups=tuned[k]["wave_groups"],
               hybrid=tuned[k]["hybrid"])
    B = fnlh.Batch(ctxs)
    use_graph = not args.no_graph
    if args.batch_loop_cells is not None:
        B.set_loop_cells(args.batch_loop_cells)
        sched = {"loop_cells": args.batch_loop_cells, "autotuned": False}
    else:
        st, pick, ms = B.autotune(systems, xd, bd, rtol=RTOL, check_every=args.check_every, use_graph=use_graph)
        sched = {"loop_cells": pick, "autotuned": True, "ms_by_loop_cells": {str(k): round(v, 1) for k, v in ms.items()}}
    tune_s = time.perf_counter() - t0
    print(f"[bench] batch autotune ({tune_s:.1f} s): contexts {tuned}, schedule {sched}", file=sys.stderr, flush=True)

    def batched(kind="dilu"):
        for row in xd:
            for x in row:
                x.zero_()
        st, reps = B.relax(systems, xd, bd, kind=kind, max_sweeps=5000, rtol=RTOL, check_every=args.check_every,
                           use_graph=use_graph, learn_every=args.learn_every)
        if st not in CONVERGED:
            raise RuntimeError(f"batched solve status {st}")
        return reps

    def loop():
        reps = []
        for c, sy, xr, br in zip(ctxs, systems, xd, bd):
            for x in xr:
                x.zero_()
            st, rep = c.relax(sy, xr, br, kind="dilu", max_sweeps=5000, rtol=RTOL, check_every=args.check_every,
                              use_graph=use_graph)
            if st not in CONVERGED:
                raise RuntimeError(f"per-instance solve status {st}")
            reps.append(rep)
        return reps

    def timeit(fn, n, w):
        for _ in range(w):
            fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(n):
            reps = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / n, reps

    tb, reps_b = timeit(batched, steps, warmup)
    print(f"[bench] batched: {1e3 * tb:.1f} ms per step", file=sys.stderr, flush=True)
    tl, reps_l = timeit(loop, max(1, steps // 2), 1)
    print(f"[bench] per-instance loop: {1e3 * tl:.1f} ms per step", file=sys.stderr, flush=True)
    # algorithmic bytes of every sweep pass of one solve of all instances (the library's
    # byte model, summed from an untimed loop with launch statistics on); the batched call
    # sweeps the same systems as often (same iterates), so the same bytes over its time
    # give its average sweep-byte rate
    for c in ctxs:
        c.stats_enable(True)
    loop()
    alg_bytes = 0
    for c in ctxs:
        alg_bytes += sum(v["alg_bytes"] for v in c.stats().values())
        c.stats_enable(False)
    learned = None
    if ckpt is not None:
        nets = [fnlh.Network(c) for c in ctxs]
        for net in nets:
            net.load(ckpt)
        tln, reps_ln = timeit(lambda: batched("learned"), max(1, steps // 2), 1)
        print(f"[bench] batched learned: {1e3 * tln:.1f} ms per step", file=sys.stderr, flush=True)
        learned = {"ms": round(1e3 * tln, 3), "vs_batched_plain": round(tb / tln, 3),
                   "sweeps_total": sum(r["sweeps"] for rep in reps_ln for r in rep),
                   "plain_sweeps_total": sum(r["sweeps"] for rep in reps_b for r in rep),
                   "learned_steps": sum(r["learned"] for rep in reps_ln for r in rep),
                   "rejected": sum(r["fallbacks"] for rep in reps_ln for r in rep),
                   "fell_back": sum(r["status"] == 3 for rep in reps_ln for r in rep),
                   "worst_rel_res": max(r["rel_res"] for rep in reps_ln for r in rep), "training": training}
        for net in nets:
            net.close()
    ncell = [c.n for c in ctxs]
    updates = sum(ncell[i] * r["sweeps"] for i, rep in enumerate(reps_b) for r in rep)
    sweeps = [r["sweeps"] for rep in reps_b for r in rep]
    out = {"workload": (f"{len(ctxs)} independent blade-row instances, {cells} cells, {n_sys_total} systems "
                        "(mean + 1-8 harmonics each), DILU to a 1e-8 residual drop, batched + graph-replayed"),
           "instances": len(ctxs), "cells": cells, "systems": n_sys_total, "storage": args.storage,
           "time_to_1e-8_ms": round(1e3 * tb, 3), "updates_per_s": round(updates / tb),
           "per_instance_loop_ms": round(1e3 * tl, 3), "batched_speedup_vs_loop": round(tl / tb, 3),
           "sweep_alg_bytes": int(alg_bytes), "sweep_alg_GBs_over_call": round(alg_bytes / tb / 1e9, 1),
           "sweep_alg_frac_over_call": round(alg_bytes / tb / 1e9 / HBM_PEAK_GBS, 4),
           "sweeps_min_max": [min(sweeps), max(sweeps)],
           "worst_rel_res": max(r["rel_res"] for rep in reps_b for r in rep),
           "autotune": {"contexts": {str(k): v for k, v in tuned.items()}, "schedule": sched,
                        "seconds": round(tune_s, 1)},
           "setup_s": round(setup_s, 1), "learned_batched": learned}
    B.close()
    for c in ctxs:
        c.close()
    return out


def run_batch(args):
    ckpt = training = None
    if not args.no_learned:
        ckpt, training = train_heldout(args.storage, [10, 11, 12, 13], args.learn_starts, 8, 4, args.learn_rounds, 8,
                                       8, 1e-3)
    res = batch_measure(args, ckpt=ckpt, training=training, warmup=args.warmup)
    out = {
        "metric": METRIC, "value": res["updates_per_s"], "unit": "cell-system-sweep updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": res["time_to_1e-8_ms"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": _dtype_of(args.storage), "data": "synthetic",
        "config": {"workload": res["workload"], "instances": res["instances"], "cells": res["cells"],
                   "systems": res["systems"], "storage": args.storage},
        "batch": res,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--storage", default="f32", choices=["f64", "f32", "bf16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-modes", action="store_true", help="skip the other storage precisions")
    ap.add_argument("--lanes", type=int, default=0, help="systems per lane of the sweep kernels (0 = auto)")
    ap.add_argument("--row-lanes", type=int, default=0, help="lanes sharing a row in the two-colour pass (0 = auto)")
    ap.add_argument("--wave-groups", type=int, default=None, choices=[0, 1],
                    help="two-colour pass: one wave per workgroup (1) or a tile per workgroup (0); default: library's")
    ap.add_argument("--check-every", type=int, default=16, help="sweeps between host checks of the stop flags")
    ap.add_argument("--no-graph", action="store_true", help="direct launches instead of graph replay")
    ap.add_argument("--no-stats", action="store_true", help="no per-kernel event timing in the timed region")
    ap.add_argument("--workload", default="largest",
                    choices=["precision", "batch", "learned", "largest", "phase", "krylov", "rk", "partition",
                             "partition_ilu"],
                    help="largest: 1.92M-cell three-row sector, mean + 10 harmonics (default); precision: 200k "
                         "cells, mean + 3 harmonics at FP64/FP32/BF16; batch: 64 uneven instances; learned: the "
                         "held-out training protocol and learned vs plain solves; phase: phase-lagged periodic "
                         "cascade; krylov: FGMRES vs "
                         "Richardson; rk: RK(5,3) pseudo-time steps around paper-mode solves; partition: RK convergence "
                         "with the couplings between partitions dropped, by partition size; partition_ilu: "
                         "partition-local natural-order ILU(0) against colour-ordered DILU, by partition size")
    ap.add_argument("--part-sizes", type=float, nargs="+", default=[16384, 4096, 1024, 256, 64],
                    help="partition workload: cells per partition (the whole mesh is always run first)")
    ap.add_argument("--max-steps", type=int, default=300, help="partition workload: pseudo-time step limit")
    ap.add_argument("--pilu-sizes", type=float, nargs="+", default=[3200, 1600, 800, 400, 200, 100, 50, 25],
                    help="partition_ilu workload: cells per partition (the whole mesh is always run first)")
    ap.add_argument("--pilu-max-sweeps", type=int, default=4000, help="partition_ilu workload: sweep limit")
    ap.add_argument("--pilu-systems", type=int, default=1,
                    help="partition_ilu workload: harmonic systems solved together (1 = the BPF)")
    ap.add_argument("--pilu-threads", type=int, default=None, choices=[0, 64, 128, 256],
                    help="partition_ilu workload: lanes per sweep workgroup of the partition-local ILU (0 = automatic)")
    ap.add_argument("--pilu-unit", type=int, default=None,
                    help="partition_ilu workload: cells per work unit of the partition-local ILU (0 = automatic)")
    ap.add_argument("--part-numbering", nargs="+", default=["structured", "random"],
                    choices=["structured", "random"], help="partition_ilu workload: cell numberings")
    ap.add_argument("--part-cfl", type=float, nargs="+", default=[50.0, 10.0], help="partition workload: CFL numbers")
    ap.add_argument("--part-kinds", nargs="+", default=["dilu", "pilu"], choices=["dilu", "pilu"],
                    help="partition workload: stage-solve preconditioners (pilu where a partition fits in LDS)")
    ap.add_argument("--restart", type=int, default=20, help="krylov workload: Krylov vectors per cycle")
    ap.add_argument("--inner-sweeps", type=int, default=1, help="krylov workload: sweeps per preconditioner application")
    ap.add_argument("--shape", type=int, nargs=3, default=list(SHAPE),
                    help="precision workload: passage cells (axial, pitch, radial); 160 100 100 gives a 1.6M-cell "
                         "working set far above the Infinity Cache")
    ap.add_argument("--largest-shape", type=int, nargs=3, default=[100, 64, 100],
                    help="largest workload: cells per row (axial, pitch, radial)")
    ap.add_argument("--pairs", type=int, default=10000, help="learned workload: training pairs")
    ap.add_argument("--train-steps", type=int, default=1250, help="learned workload: Adam steps")
    ap.add_argument("--batch", type=int, default=8, help="learned workload: pairs per Adam step")
    ap.add_argument("--learn-every", type=int, default=32, help="sweeps between learned corrections")
    ap.add_argument("--no-learned", action="store_true", help="skip the short learned-vs-plain comparison")
    ap.add_argument("--no-batch", action="store_true", help="largest workload: skip the 64-instance batching field")
    ap.add_argument("--hybrid", type=int, default=1, choices=[0, 1, 2],
                    help="multi-colour orderings: 1 two-colour + remainder passes when the remainder is small "
                         "(default), 0 general passes, 2 always two-colour + remainder")
    ap.add_argument("--learn-starts", type=int, default=16,
                    help="largest workload: random starts per system and training mesh (8 snapshots each)")
    ap.add_argument("--learn-rounds", type=int, default=15,
                    help="largest workload: training rounds (8 Adam steps on each of the 4 meshes per round)")
    ap.add_argument("--instances", type=int, default=64)
    ap.add_argument("--batch-loop-cells", type=int, default=None,
                    help="batch workload: instances of at least this many cells are iterated alone inside the "
                         "batched call (0: all batched; default: the library's, 80k cells)")
    ap.add_argument("--total-cells", type=float, default=8.0e6)
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 1 GiB read + 1 GiB write elementwise kernel (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (no multi-GPU path); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.workload == "largest":
        return run_largest(args)  # initialises the GPU after its CPU oracle sample
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.workload == "batch":
        return run_batch(args)
    if args.workload == "learned":
        return run_learned(args)
    if args.workload == "phase":
        return run_phase(args)
    if args.workload == "krylov":
        return run_krylov(args)
    if args.workload == "rk":
        return run_rk(args)
    if args.workload == "partition":
        return run_partition(args)
    if args.workload == "partition_ilu":
        return run_partition_ilu(args)

    if args.calib_copy:
        calib_copy()

    mesh, Q, om, bs = build_inputs(tuple(args.shape))
    print(f"[bench] inputs: {mesh.n_cells} cells, {mesh.n_edges} faces, {len(bs)} systems", file=sys.stderr, flush=True)
    main_run = Runner(mesh, Q, om, bs, args.storage, args.lanes, args.row_lanes, args.check_every,
                      not args.no_graph, args.wave_groups)
    res = main_run.timed(args.steps, args.warmup, stats=not args.no_stats)
    print(f"[bench] {args.storage}: {res['ms_per_step']:.2f} ms/step, sweeps {res['sweeps']}", file=sys.stderr,
          flush=True)
    st = res["stats"] or {k: {"launches": 0, "total_ms": 0.0, "alg_bytes": 0.0} for k in ("sweep_update", "sweep_set")}
    upd = st["sweep_update"]
    setp = st["sweep_set"]
    avg_ms = upd["total_ms"] / max(upd["launches"], 1)
    bytes_per_launch = upd["alg_bytes"] / max(upd["launches"], 1)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    traffic, traffic_src = None, "not measured for a tuned kernel shape"
    if args.lanes == 0 and args.row_lanes == 0:
        traffic, traffic_src = traffic_from_profile(precision_profile_name(args.storage, mesh.n_cells))
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "traffic_source": traffic_src,
                "kernel": f"k_rb_pass<{args.storage}, update> (two-colour sweep pass over the second colour)",
                "avg_launch_us": round(1e3 * avg_ms, 2), "alg_bytes_per_launch": round(bytes_per_launch),
                "launches": upd["launches"]}
    if setp["launches"]:
        set_ms = setp["total_ms"] / setp["launches"]
        roofline["other_pass"] = {
            "kernel": "k_rb_pass<set> (first colour)", "avg_launch_us": round(1e3 * set_ms, 2),
            "achieved": round(setp["alg_bytes"] / setp["launches"] / (set_ms * 1e-3) / 1e9, 1)}
    memory = main_run.ctx.memory()
    colour, _ = main_run.ctx.ordering()

    modes = {}
    if not args.no_modes:
        sols = {args.storage: [x.clone() for x in main_run.xd]}
        for s in ("f64", "f32", "bf16"):
            if s == args.storage:
                continue
            r = Runner(mesh, Q, om, bs, s, check_every=args.check_every, use_graph=not args.no_graph)
            m = r.timed(3, 1)
            sols[s] = [x.clone() for x in r.xd]
            modes[s] = {"ms_per_step": round(m["ms_per_step"], 3), "updates_per_s": round(m["updates_per_s"]),
                        "sweeps": m["sweeps"], "outer": m["outer"], "rel_res": m["rel_res"]}
            r.ctx.close()
            print(f"[bench] {s}: {m['ms_per_step']:.2f} ms/step, sweeps {m['sweeps']}", file=sys.stderr, flush=True)
        # error of each precision's solution against the FP64 one (the FP64 path is held
        # to the oracle by the parity tests)
        for s, xs in sols.items():
            err = [float(torch.linalg.norm(a - b) / torch.linalg.norm(b)) for a, b in zip(xs, sols["f64"])]
            if s == args.storage:
                res["err_vs_f64"] = err
            else:
                modes[s]["err_vs_f64"] = err

    learned = None
    if not args.no_learned:
        print("[bench] short learned-vs-plain comparison (512 pairs, 128 Adam steps)", file=sys.stderr, flush=True)
        learned = learned_compare(mesh, Q, om, bs, args.storage, 512, 128, 8, args.learn_every)
        print(f"[bench] learned: plain {learned['plain']['ms']} ms, learned {learned['learned']['ms']} ms",
              file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle sample", file=sys.stderr, flush=True)
        cpu = cpu_baseline(mesh, Q, om, bs, colour, res["sweeps"])

    out = {
        "metric": METRIC,
        "value": round(res["updates_per_s"]),
        "unit": "cell-unknown updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(res["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": _dtype_of(args.storage),
        "data": "synthetic",
        "config": {"workload": (f"{mesh.n_cells}-cell hex annular passage sector {'x'.join(map(str, args.shape))} "
                                f"({mesh.n_edges} faces), mean + 3 harmonics (omega = 0, 18, 36, 54), "
                                "DILU-preconditioned Richardson to a 1e-8 residual drop"),
                   "cells": mesh.n_cells, "faces": mesh.n_edges, "systems": len(bs), "storage": args.storage,
                   "eps": 0.6, "sigma": 50.0},
        "time_to_1e-8_ms": round(res["ms_per_step"], 3),
        "sweeps": res["sweeps"],
        "outer": res["outer"],
        "rel_res": res["rel_res"],
        "err_vs_f64": res.get("err_vs_f64"),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "modes": modes,
        "learned": learned,
        "memory_bytes": memory,
        "ingest_ms": round(main_run.ingest_ms, 1),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
