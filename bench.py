#!/usr/bin/env python
"""Damped-gradient iterations per second of the 48^3 x 2000-nucleon pasta box.

One step = one full static iteration (Fig. 1 steps 2-5 of the paper) for
both species, in the mixed-precision form by default (complex64 states, FP32
FFTs and h psi, split-FP16 MFMA GEMMs, FP64 subspace solve), with the FP64
form timed on the same box for comparison: h psi, damped gradient step, h phi, overlap and subspace
Hamiltonian GEMMs, Cholesky + Jacobi Rayleigh-Ritz, recombination GEMM,
densities, mean field, Coulomb and energy.  Inputs are synthetic (seeded
rod-perturbed plane waves, SLy4) and already resident in HBM when the timed
region starts.  Prints one JSON line.

The roofline entry is for the kernel with the most device time, timed with
HIP events on the library's own stream; cpu_baseline is the FP64 numpy
oracle timed on a bounded sample of the same iteration and scaled to a full
iteration.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6      # MI355X dense FP64 (matrix and vector)
PEAK_F16_TFLOPS = 2500.0     # MI355X dense FP16 / BF16 matrix
PEAK_HBM_GBS = 8000.0        # MI355X HBM3E
SPLIT_PRODUCTS = 3           # FP16 products per real product in the mixed GEMMs


# HBM bytes per neutron launch of the roofline kernels on the 48^3 x 1600
# neutron box, from rocprofv3 --pmc runs of this script (FETCH_SIZE, then
# WRITE_SIZE, in KiB per dispatch), scaled by what the same counters read for
# a 1 GiB device copy (FETCH_SIZE x2, WRITE_SIZE x1).  A figure is reported
# only while the kernel's source file still has the hash it was measured on.
MEASURED_TRAFFIC = {
    "k_overlap_planes": dict(fetch_kib=1.40552e7, write_kib=745472.0, fetch_scale=2.0,
                             write_scale=1.0, source="paper_1610_07522_amd/csrc/k_gemm_mixed.hip",
                             sha256_16="3a31b06841365034"),
    "k_combine_planes": dict(fetch_kib=1.00463e7, write_kib=2764800.0, fetch_scale=2.0,
                             write_scale=1.0, source="paper_1610_07522_amd/csrc/k_gemm_mixed.hip",
                             sha256_16="3a31b06841365034"),
}


# HBM bytes per neutron launch of each grid phase, summed over its kernels
# (rocprofv3 FETCH_SIZE x2 + WRITE_SIZE, profiles/grid_kernels_rod48_pmc.md),
# reported while k_grid.hip keeps the hash they were taken on.
MEASURED_PHASE_TRAFFIC = dict(
    source="paper_1610_07522_amd/csrc/k_grid.hip", sha256_16="d6d130e6e9b5ffa4",
    apply_h=22.662e9, damp=22.654e9, densities=9.402e9)


def measured_phase_traffic(phase: str):
    import hashlib
    e = MEASURED_PHASE_TRAFFIC
    with open(os.path.join(ROOT, e["source"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest()[:16] != e["sha256_16"]:
            return None
    return e.get(phase)


def measured_traffic(kernel: str):
    """Bytes per launch from MEASURED_TRAFFIC, or None if not measured or stale."""
    import hashlib
    e = MEASURED_TRAFFIC.get(kernel)
    if e is None:
        return None
    with open(os.path.join(ROOT, e["source"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest()[:16] != e["sha256_16"]:
            return None
    return 1024.0 * (e["fetch_kib"] * e["fetch_scale"] + e["write_kib"] * e["write_scale"])


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def gemm_flops(m: int, v: int) -> dict:
    """Algorithmic real flops per launch: complex MAC = 8 flops.
    overlap: I and H lower triangles incl. diagonal; combine: psi = phi U."""
    return dict(overlap_gemm=8.0 * 2 * (m * (m + 1) // 2) * v,
                combine_gemm=8.0 * m * m * v)


def roofline(timing: dict, w, mixed: bool) -> dict:
    """Roofline of the costlier of the two single-kernel GEMM phases (the
    I/H overlap GEMM or the recombination GEMM), neutron launches.  achieved
    counts the method's own arithmetic, 8 real flops per complex
    multiply-add of the contraction (lower triangles of I and H), against
    the peak of the dtype the kernel runs on: FP64 MFMA for the FP64 form,
    FP16 MFMA for the mixed form.  The split-FP16 kernel issues 3 FP16
    products per real product; that issue rate is reported separately
    ("issued") and is not counted as work."""
    v = 2 * w.n ** 3
    m = w.n_neutrons
    dom = max(("overlap_gemm", "combine_gemm"),
              key=lambda k: timing[k]["ms_n"] + timing[k]["ms_p"])
    t = timing[dom]
    avg_ms = t["ms_n"] / max(1, t["launches_n"])
    fl = gemm_flops(m, v)[dom]
    peak = PEAK_F16_TFLOPS if mixed else PEAK_FP64_TFLOPS
    ach = fl / (avg_ms * 1e-3) / 1e12
    if mixed:
        name = "k_overlap_planes" if dom == "overlap_gemm" else "k_combine_planes"
    else:
        name = "k_overlap_lower" if dom == "overlap_gemm" else "k_combine"
    traffic = measured_traffic(name) if w.name == "rod48" else None
    out = dict(kernel=name, bound="mfma", achieved=ach, peak=peak, unit="TFLOP/s",
               frac=ach / peak, traffic=traffic, traffic_unit="bytes per launch",
               dtype=("fp16 MFMA (two-term split of c64 operands)" if mixed else "fp64"),
               per_launch=dict(species="neutrons", m=m, k=v, flops=fl, avg_ms=avg_ms,
                               unique_bytes=2.0 * m * v * (8 if mixed else 16)))
    if mixed:
        iss = ach * SPLIT_PRODUCTS
        out["issued"] = dict(achieved=iss, frac=iss / peak, unit="TFLOP/s",
                             note=f"{SPLIT_PRODUCTS} FP16 products per real product of the split")
    return out


# HBM bytes a phase must move per launch per state (complex elements V = 2 n^3
# per state): h psi reads psi and writes h psi; the damped step reads psi and
# h psi and writes phi; the densities read psi.
PHASE_STATE_ARRAYS = dict(apply_h=2, damp=3, densities=1)


def hbm_phases(timing: dict, w, mixed: bool) -> dict:
    """Algorithmic HBM rate of each grid phase (neutron launches): compulsory
    bytes (PHASE_STATE_ARRAYS state arrays) / the phase's mean launch time."""
    v = 2 * w.n ** 3
    m = w.n_neutrons
    out = {}
    for ph_, arrays in PHASE_STATE_ARRAYS.items():
        t = timing[ph_]
        if not t["launches_n"]:
            continue
        avg_ms = t["ms_n"] / t["launches_n"]
        nbytes = arrays * m * v * (8 if mixed else 16)
        ach = nbytes / (avg_ms * 1e-3) / 1e9
        out[ph_] = dict(achieved=ach, frac=ach / PEAK_HBM_GBS, avg_ms=avg_ms,
                        bytes_per_launch=nbytes, state_arrays=arrays)
        cb = measured_phase_traffic(ph_) if (mixed and w.name == "rod48") else None
        if cb is not None:
            out[ph_]["counter_bytes"] = cb
            out[ph_]["counter_achieved"] = cb / (avg_ms * 1e-3) / 1e9
            out[ph_]["counter_frac"] = out[ph_]["counter_achieved"] / PEAK_HBM_GBS
    out["unit"] = "GB/s"
    out["peak"] = PEAK_HBM_GBS
    return out


def h_phase_hbm(timing: dict, w, mixed: bool) -> dict:
    """Algorithmic HBM rate of one h*psi application (read psi, write h psi),
    neutron launches."""
    v = 2 * w.n ** 3
    m = w.n_neutrons
    t = timing["apply_h"]
    avg_ms = t["ms_n"] / max(1, t["launches_n"])
    nbytes = 2.0 * m * v * (8 if mixed else 16)
    ach = nbytes / (avg_ms * 1e-3) / 1e9
    return dict(phase="apply_h", bound="hbm", achieved=ach, peak=PEAK_HBM_GBS,
                unit="GB/s", frac=ach / PEAK_HBM_GBS, bytes_per_launch=nbytes, avg_ms=avg_ms)


def oracle_config0(iters: int = 200) -> dict:
    """The oracle measured in full (not sampled) on the 16^3 box with
    8 n + 8 p: init plus ``iters`` iterations."""
    from threadpoolctl import threadpool_limits

    from oracle import Grid
    from oracle import solver as so
    from paper_1610_07522_amd import inputs

    cores = int(os.environ.get("SKY_ORACLE_THREADS", "0")) or len(os.sched_getaffinity(0))
    os.environ["SKY_ORACLE_THREADS"] = str(cores)
    w = inputs.WORKLOADS["fermi16"]
    raw = inputs.raw_states(w)
    with threadpool_limits(limits=cores):
        t0 = time.perf_counter()
        st = so.initial_state(*raw, Grid(w.n, w.dx), w.params, w.damp_x0, w.damp_e0)
        t_init = time.perf_counter() - t0
        t0 = time.perf_counter()
        for _ in range(iters):
            rep = so.iterate(st)
        sec = time.perf_counter() - t0
    return dict(workload="fermi16: 16^3, 8 n + 8 p, plane waves + noise 0.1", iterations=iters,
                seconds=sec, iter_per_s=iters / sec, init_seconds=t_init,
                residual_after=rep.de, energy_after=rep.E["total"], cores=cores)


def cpu_baseline(w, budget_states: int = 8, k_slice: int = 32) -> dict:
    """FP64 oracle on the host, bounded sample, scaled to one full iteration.

    Per-state work (h psi twice, damping, densities) is timed on
    ``budget_states`` states per species and scaled by N_q / budget; the
    overlap/H and recombination products on 1/k_slice of the grid
    (contraction length) and scaled by k_slice; mean field and the dense
    Rayleigh-Ritz (Cholesky, eigh) of both species run in full.
    """
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import Grid
    from oracle import physics as ph
    from oracle import solver as so
    from paper_1610_07522_amd import inputs

    cores = int(os.environ.get("SKY_ORACLE_THREADS", "0")) or len(os.sched_getaffinity(0))
    os.environ["SKY_ORACLE_THREADS"] = str(cores)
    g = Grid(w.n, w.dx)
    v = 2 * w.n ** 3
    sub = inputs.Workload("sample", w.n, w.dx, budget_states, budget_states, w.init,
                          seed=w.seed, amp=w.amp, noise=w.noise)
    rn, rp = inputs.raw_states(sub)
    t = {}
    with threadpool_limits(limits=cores):
        t0 = time.perf_counter()
        dn, dp = ph.densities(rn, g), ph.densities(rp, g)
        t["densities"] = (time.perf_counter() - t0) * w.n_states / (2 * budget_states)
        t0 = time.perf_counter()
        mn, mp, vc = ph.mean_field(dn, dp, g, w.params)
        ph.energy(dn, dp, g, w.params, vc)
        t["meanfield"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        for raw, mf in ((rn, mn), (rp, mp)):
            h = ph.apply_h(raw, mf, g)
            eps, r, _ = so.rayleigh_and_residual(raw, h, g)
            phi = raw - so.damping(r, g, mf.hb2m, w.damp_x0, w.damp_e0)
            ph.apply_h(phi, mf, g)
        t["per_state"] = (time.perf_counter() - t0) * w.n_states / (2 * budget_states)
        rng = np.random.default_rng(0)
        kk = v // k_slice
        t_gemm = 0.0
        t_rr = 0.0
        for m in (w.n_neutrons, w.n_protons):
            a = rng.standard_normal((m, kk)) + 1j * rng.standard_normal((m, kk))
            b = rng.standard_normal((m, kk)) + 1j * rng.standard_normal((m, kk))
            t0 = time.perf_counter()
            I = g.dV * (a.conj() @ a.T)
            H = g.dV * (a.conj() @ b.T)
            U = np.eye(m, dtype=complex) + 1e-3 * I / max(1.0, abs(I).max())
            (U.T @ a)
            t_gemm += (time.perf_counter() - t0) * k_slice
            Ih = a.conj() @ a.T / kk + np.eye(m)
            Hh = 0.5 * (H + H.conj().T)
            t0 = time.perf_counter()
            so.rayleigh_ritz(Ih, Hh)
            t_rr += time.perf_counter() - t0
        t["gemm"] = t_gemm
        t["rayleigh_ritz"] = t_rr
    sec = sum(t.values())
    sample = (f"{budget_states}+{budget_states} states for the per-state phases (scaled x"
              f"{w.n_states / (2 * budget_states):.0f}), 1/{k_slice} of the grid for the "
              f"overlap/H/recombination products (scaled x{k_slice}), full mean field and "
              f"full dense Rayleigh-Ritz of both species; est. {sec:.1f} s per iteration")
    return dict(value=1.0 / sec, unit="iter/s", cores=cores, kind="oracle", sample=sample,
                seconds_per_iter=sec, parts_s={k: round(x, 3) for k, x in t.items()})


def copy_bandwidth(dev) -> dict:
    """Measured device-to-device copy rate (1 GiB, read + write counted), the
    practical ceiling for the HBM-bound phases next to the 8 TB/s peak."""
    import torch
    src = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(10):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    sec = a.elapsed_time(b) / 1e3 / 10
    gbs = 2.0 * (4 << 28) / sec / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return dict(achieved=gbs, peak=PEAK_HBM_GBS, unit="GB/s", frac=gbs / PEAK_HBM_GBS,
                note="torch device copy of 1 GiB, bytes read + written")


def workload_of(args):
    """The named workload with the requested extra states (a fraction of each
    species' particles, rounded up)."""
    import dataclasses

    from paper_1610_07522_amd import inputs
    w = inputs.WORKLOADS[args.workload]
    if args.extra > 0:
        w = dataclasses.replace(w, extra_n=math.ceil(args.extra * w.n_neutrons),
                                extra_p=math.ceil(args.extra * w.n_protons))
    return w


def form_kwargs(args) -> dict:
    """Descriptor options of the iteration form chosen on the command line."""
    from paper_1610_07522_amd import inputs, sky
    kw = dict(update=sky.SKY_UPDATE_PAPER if args.update == "paper" else sky.SKY_UPDATE_EXACT,
              one_h=args.one_h)
    if args.twists > 1:
        kw["twists"] = inputs.special_twists(args.twists)
    return kw


def form_config(args, w) -> dict:
    return dict(extra_states=[w.extra_n, w.extra_p], update=args.update, one_h=args.one_h,
                twists=(args.twists ** 3 if args.twists > 1 else 1))


def bench_batch(args) -> int:
    """64 independent uneven boxes (16^3-32^3, 102-512 nucleons, mixed
    precision): box-iterations per second of the batched driver with the
    device-decided iteration graphs (worker threads with their own streams,
    one host synchronisation per worker per chunk), beside the batched
    driver with host-decided subspace solves and the same boxes iterated one
    after another on one stream without graphs."""
    import torch

    from paper_1610_07522_amd import inputs, sky

    ws = inputs.batch_workloads(64)
    dev = torch.device("cuda:0")
    boxes = []
    t0 = time.perf_counter()
    for w in ws:
        d = sky.desc_from_workload(w, precision=sky.SKY_MIXED)
        d.dev_refine_steps = args.dev_refine_steps
        b = sky.Box(d, device=dev)
        rn, rp = inputs.raw_states(w)
        dn, dp = torch.from_numpy(rn).to(dev), torch.from_numpy(rp).to(dev)
        del rn, rp
        b.init_box(dn, dp)
        if args.tune_cache != "off":
            b.autotune(args.tune_cache)
            b.init_box(dn, dp)
        del dn, dp
        boxes.append(b)
    torch.cuda.synchronize()
    log(f"64 boxes initialised in {time.perf_counter() - t0:.1f} s "
        f"(workspaces {sum(b.nbytes for b in boxes) / 1e9:.1f} GB)")
    k = args.steps
    chunk = min(k, 16)
    reps = sky.batch_iterate(boxes, args.threads, args.warmup)   # captures the graphs
    reps = sky.batch_iterate_graph(boxes, args.threads, args.warmup, 0.0, chunk)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for b in boxes:
        b.iterate(k)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    log(f"one stream, no graphs: {64 * k} box-iterations in {t_seq:.3f} s")
    t0 = time.perf_counter()
    reps = sky.batch_iterate(boxes, args.threads, k)
    torch.cuda.synchronize()
    t_bat = time.perf_counter() - t0
    log(f"batched ({args.threads} workers, graphs, host-decided solve): {64 * k} box-iterations "
        f"in {t_bat:.3f} s")
    t0 = time.perf_counter()
    reps = sky.batch_iterate_graph(boxes, args.threads, k, 0.0, chunk)
    torch.cuda.synchronize()
    t_dev = time.perf_counter() - t0
    handovers = sum(r["eig_fallbacks"] for r in reps)
    log(f"batched ({args.threads} workers, device-decided iteration graphs, chunks of {chunk}): "
        f"{64 * k} box-iterations in {t_dev:.3f} s; {handovers} iterations finished on the host")
    grids = sorted({w.n for w in ws})
    out = dict(
        metric="box-iterations/s, 64 independent uneven boxes",
        value=64 * k / t_dev, unit="box-iter/s", n_gpus=1, steps=k, warmup=args.warmup,
        ms_per_step=1e3 * t_dev / k, higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype="mixed: c64 states, f32 FFT/h*psi, fp16x2-split MFMA GEMMs, f64 subspace solve",
        data="synthetic",
        config=dict(workload=(f"64 boxes, grids {grids} at 1 fm, "
                              f"{min(w.n_states for w in ws)}-{max(w.n_states for w in ws)} "
                              "nucleons, proton fraction 0.1-0.5, density 0.02-0.06 fm^-3, "
                              "slab/rod/random starts, SLy4"),
                    boxes=64, workers=args.threads, chunk=chunk,
                    driver="sky_batch_iterate_graph (device-decided iteration graphs)"),
        handovers=handovers,
        dev_refine_steps=args.dev_refine_steps or 4,
        host_decided=dict(value=64 * k / t_bat, unit="box-iter/s",
                          note="sky_batch_iterate: graph segments, subspace solve and "
                               "residual decided on the host every iteration"),
        sequential=dict(value=64 * k / t_seq, unit="box-iter/s",
                        note="same boxes one after another, one stream, eager launches"),
        speedup=t_seq / t_dev,
        residual_range=[min(r["residual"] for r in reps), max(r["residual"] for r in reps)],
    )
    print(json.dumps(out), flush=True)
    return 0


def bench_mlp(args) -> int:
    """Training steps of the learned damping's MLP (sky_precond_loss_grad) on
    args.mlp_rows seeded synthetic rows: features in the ranges the learned
    step produces, targets and weights; the network as sky_init_box sets it."""
    import numpy as np
    import torch
    from paper_1610_07522_amd import inputs, sky
    B = args.mlp_rows
    w = inputs.small_workload("n8", 8, 5, 3, init="slab", seed=32, noise=0.2)
    box = sky.Box(sky.desc_from_workload(w, precision=sky.SKY_FP64))
    rn, rp = inputs.raw_states(w)
    box.init_box(torch.from_numpy(rn).cuda(), torch.from_numpy(rp).cuda())
    cap = box.view("pc_samples").shape[0]
    if B > cap:
        print(f"--mlp-rows at most {cap}", file=sys.stderr)
        return 2
    rng = np.random.default_rng(7)
    rows = np.zeros((B, 6), dtype=np.float32)
    rows[:, 0] = (rng.integers(0, 8, B) + 0.5) / 8      # shell centre |k| / |k|max
    rows[:, 1] = rng.uniform(-0.6, 0.1, B)              # <h> / E0
    rows[:, 2] = rng.uniform(-1, 1, B)                  # shell power share (log scale)
    rows[:, 3] = rng.uniform(0, 8, B)                   # T_k / E0
    rows[:, 4] = rng.uniform(0, 4, B)                   # target gain
    rows[:, 5] = rng.uniform(0, 1, B)                   # weight
    box.view("pc_samples")[:B].copy_(torch.from_numpy(rows).cuda())
    for _ in range(args.warmup):
        box.precond_loss_grad(B)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        loss = box.precond_loss_grad(B)
    dt = time.perf_counter() - t0
    print(json.dumps(dict(metric="learned-damping MLP training step (forward, loss, backward, gradient)",
                          rows=B, steps=args.steps, ms_per_step=1e3 * dt / args.steps,
                          loss=loss, note="host time per step includes one synchronisation")),
          flush=True)
    return 0


def bench_learned_protocol(args) -> int:
    """The learned damping trained on other boxes and judged on held-out
    ones.  Training: for seeds 100-131, the three box shapes of the 16^3
    (8 n + 8 p, noise 0.1), 32^3 slab (640 n + 160 p) and 48^3 rod
    (1600 n + 400 p) workloads are each iterated a few times in the mixed
    form, rows are collected from both species and the network takes Adam
    steps on them; the network is carried from box to box with
    sky_set_preconditioner (Adam moments restart per box).  Evaluation: the
    48^3 rod box with the held-out seeds 200-203, from the same states, plain
    damping against the carried network (no further training), iterations
    and wall time until Delta-eps <= tol (tested from min_iter on)."""
    import dataclasses

    import numpy as np
    import torch

    from paper_1610_07522_amd import inputs, sky

    dev = torch.device("cuda:0")
    shapes = [(inputs.WORKLOADS["fermi16"], 20), (inputs.WORKLOADS["slab32"], 30),
              (inputs.WORKLOADS["rod48"], 30)]
    params = None
    t0 = time.perf_counter()
    losses = [float("nan")]
    if args.params_in:
        params = torch.from_numpy(np.load(args.params_in)).to(dev)
        log(f"network loaded from {args.params_in}")
    for seed in (range(100, 132) if not args.params_in else ()):
        for base, warm in shapes:
            w = dataclasses.replace(base, seed=seed)
            rn, rp = inputs.raw_states(w)
            box = sky.Box(sky.desc_from_workload(w, precision=sky.SKY_MIXED), device=dev)
            box.init_box(torch.from_numpy(rn).to(dev), torch.from_numpy(rp).to(dev))
            del rn, rp
            if params is not None:
                box.set_preconditioner(params)
            box.iterate(warm)
            for q in range(2):
                box.precond_collect(q)
            losses.append(box.precond_train(args.train_steps, 1e-3))
            params = box.view("pc_params").clone()
            box.close()
            del box
            torch.cuda.empty_cache()
        log(f"training: seeds 100-{seed} done, loss {losses[-1]:.4e}, "
            f"{time.perf_counter() - t0:.0f} s")
    t_train = time.perf_counter() - t0
    if args.params_out:
        np.save(args.params_out, params.cpu().numpy())
        log(f"network saved to {args.params_out}")
    tol = args.to_residual if args.to_residual > 0 else 0.1
    evals = []
    first = min(max(args.eval_from, 200), 203)
    for seed in range(first, min(first + max(args.eval_seeds, 0), 204)):
        w = dataclasses.replace(inputs.WORKLOADS["rod48"], seed=seed)
        rn, rp = inputs.raw_states(w)
        dn, dp = torch.from_numpy(rn).to(dev), torch.from_numpy(rp).to(dev)
        del rn, rp
        row = dict(seed=seed)
        for mode in ("plain", "learned"):
            box = sky.Box(sky.desc_from_workload(w, precision=sky.SKY_MIXED), device=dev)
            box.init_box(dn, dp)
            if args.tune_cache != "off":
                box.autotune(args.tune_cache)
                box.init_box(dn, dp)
            if mode == "learned":
                box.set_preconditioner(params)
                box.precond_use(True, 0.05, 0)
            torch.cuda.synchronize()
            ts = time.perf_counter()
            its, rep, shown = 0, None, ts
            while its < args.max_iter:
                armed = its >= args.min_iter
                chunk = min(100, args.max_iter - its) if armed else min(100, args.min_iter - its)
                rep = box.iterate(chunk, tol if armed else 0.0)
                its += rep["iters"]
                if armed and rep["converged"]:
                    break
                if time.perf_counter() - shown > 30:
                    shown = time.perf_counter()
                    log(f"eval seed {seed} {mode}: iteration {its}, residual {rep['residual']:.3e}")
            torch.cuda.synchronize()
            row[mode] = dict(iterations=its, seconds=time.perf_counter() - ts,
                             converged=bool(rep["converged"]), residual=rep["residual"],
                             energy=rep["energy"])
            log(f"eval seed {seed} {mode}: {its} iterations, {row[mode]['seconds']:.1f} s, "
                f"residual {rep['residual']:.3e}")
            box.close()
            del box
            torch.cuda.empty_cache()
        evals.append(row)
    out = dict(metric=f"learned damping trained on other boxes: time to residual {tol:g}, "
                      "48^3 rod box, held-out seeds",
               train=dict(seeds="100-131", boxes=3 * 32, shapes=[s[0].name for s in shapes],
                          warm_iterations=[s[1] for s in shapes], adam_steps_per_box=args.train_steps,
                          seconds=t_train, last_loss=losses[-1],
                          loaded_from=args.params_in or None),
               tol=tol, min_iter=args.min_iter, max_iter=args.max_iter, evaluation=evals)
    done = [e for e in evals if e["plain"]["converged"] and e["learned"]["converged"]]
    if done:
        out["mean_iterations_ratio"] = sum(e["plain"]["iterations"] / e["learned"]["iterations"]
                                           for e in done) / len(done)
        out["mean_time_ratio"] = sum(e["plain"]["seconds"] / e["learned"]["seconds"]
                                     for e in done) / len(done)
    print(json.dumps(out), flush=True)
    return 0


def bench_to_residual(args) -> int:
    """Iterations and wall time until Delta-eps <= tol on one workload, for
    the mixed form, the FP64 form and the mixed form with the learned damping
    (its sample collection and training counted in its time)."""
    import torch

    from paper_1610_07522_amd import inputs, sky

    w = workload_of(args)
    dev = torch.device("cuda:0")
    rn, rp = inputs.raw_states(w)
    dn, dp = torch.from_numpy(rn).to(dev), torch.from_numpy(rp).to(dev)
    del rn, rp
    tol = args.to_residual
    results = {}
    t_start = time.perf_counter()
    for mode in args.modes.split(","):
        prec = sky.SKY_FP64 if mode == "fp64" else sky.SKY_MIXED
        ladder = args.ladder if prec == sky.SKY_MIXED else 0.0
        box = sky.Box(sky.desc_from_workload(w, precision=prec, ladder_tol=ladder,
                                             **form_kwargs(args)), device=dev)
        box.init_box(dn, dp)
        if args.tune_cache != "off":
            box.autotune(args.tune_cache)
            box.init_box(dn, dp)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its, pc_its, rep = 0, 0, None
        if mode == "learned":
            rep = box.iterate(20)
            its += 20
            for _ in range(6):
                box.precond_collect(0)
                box.precond_collect(1)
                rep = box.iterate(5)
                its += 5
            box.precond_collect(0)
            box.precond_train(300, 1e-3)
            box.precond_use(True, 0.05, 100)
        traj = []
        while its < args.max_iter:
            # the tolerance counts from min_iter on: before the pasta structure has
            # formed, Delta-eps dips below it and rises again
            armed = its >= args.min_iter
            chunk = min(100, args.max_iter - its) if armed else min(100, args.min_iter - its)
            rep = box.iterate(chunk, tol if armed else 0.0)
            its += rep["iters"]
            pc_its += rep["precond_iters"]
            traj.append([its, round(rep["residual"], 6), round(rep["energy"], 4)])
            log(f"[{mode}] {its} iterations, residual {rep['residual']:.4e}, "
                f"E {rep['energy']:.6f}, {time.perf_counter() - t0:.1f} s")
            if armed and rep["converged"]:
                break
            if args.max_seconds > 0 and time.perf_counter() - t_start > args.max_seconds:
                log(f"[{mode}] stopped at the wall-time cap of {args.max_seconds:.0f} s")
                break
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        ritz = [box.view("ritz", q).cpu().tolist() for q in range(2)]
        results[mode] = dict(iterations=its, seconds=sec,
                             converged=bool(rep["converged"] and rep["residual"] <= tol),
                             residual=rep["residual"], energy=rep["energy"],
                             precision_at_end="fp64" if rep["precision"] == 0 else "mixed",
                             learned_iterations=pc_its, trajectory=traj, ritz=ritz)
        box.close()
        del box
        torch.cuda.empty_cache()
    out = dict(metric=f"time to residual {tol:g}", workload=w.name, tol=tol,
               min_iter=args.min_iter, max_iter=args.max_iter, ladder=args.ladder,
               form=form_config(args, w), results=results)
    if "mixed" in results and "fp64" in results:
        out["fp64_over_mixed_time"] = results["fp64"]["seconds"] / results["mixed"]["seconds"]
    if "mixed" in results and "learned" in results:
        out["plain_over_learned_time"] = results["mixed"]["seconds"] / results["learned"]["seconds"]
    if "fp64" in results:
        import numpy as np
        ref = results["fp64"]
        for k, v in results.items():
            if k == "fp64":
                continue
            v["energy_rel_diff_vs_fp64"] = abs(v["energy"] - ref["energy"]) / abs(ref["energy"])
            v["max_sp_energy_diff_vs_fp64_MeV"] = max(
                float(np.max(np.abs(np.sort(a) - np.sort(b)))) if len(a) else 0.0
                for a, b in zip(v["ritz"], ref["ritz"]))
    for v in results.values():
        v.pop("ritz")
    print(json.dumps(out), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rod48")
    ap.add_argument("--precision", choices=("mixed", "fp64"), default="mixed")
    ap.add_argument("--no-fp64-compare", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_1610_07522_amd",
                                                         "tuning_mi355x.json"),
                    help="autotuner cache (launch shapes); 'off' keeps the defaults")
    ap.add_argument("--threads", type=int, default=16,
                    help="host workers of the batched driver (workload batch64)")
    ap.add_argument("--dev-refine-steps", type=int, default=0,
                    help="workload batch64: refinement steps of the device-decided iteration "
                         "before a set is handed to the host (0: the library default)")
    ap.add_argument("--to-residual", type=float, default=0.0,
                    help="instead of iterations/s: iterations and time until Delta-eps <= this")
    ap.add_argument("--modes", default="mixed,fp64,learned",
                    help="forms run by --to-residual (mixed, fp64, learned)")
    ap.add_argument("--max-iter", type=int, default=4000)
    ap.add_argument("--min-iter", type=int, default=0,
                    help="--to-residual: the tolerance is tested from this iteration on")
    ap.add_argument("--ladder", type=float, default=0.0,
                    help="--to-residual: mixed forms switch to FP64 at this Delta-eps (0: never)")
    ap.add_argument("--extra", type=float, default=0.0,
                    help="extra unoccupied states per species, as a fraction of its particles")
    ap.add_argument("--twists", type=int, default=1,
                    help="k: twist-averaged boundary conditions over the k^3 special twists")
    ap.add_argument("--update", choices=("exact", "paper"), default="exact",
                    help="subspace update: exact Rayleigh-Ritz or the paper-literal Z C")
    ap.add_argument("--one-h", action="store_true",
                    help="one h application per iteration (h psi carried through the update)")
    ap.add_argument("--train-steps", type=int, default=20,
                    help="--workload learned_protocol: Adam steps per training box")
    ap.add_argument("--params-out", default="",
                    help="--workload learned_protocol: save the trained network (.npy)")
    ap.add_argument("--params-in", default="",
                    help="--workload learned_protocol: skip training, load this network")
    ap.add_argument("--eval-seeds", type=int, default=4,
                    help="--workload learned_protocol: held-out seeds evaluated (0-4)")
    ap.add_argument("--eval-from", type=int, default=200,
                    help="--workload learned_protocol: first held-out seed (200-203)")
    ap.add_argument("--max-seconds", type=float, default=0.0,
                    help="--to-residual: stop every form once this much wall time has passed")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run three 1 GiB device-to-device copies (HBM counter scale)")
    ap.add_argument("--mlp-rows", type=int, default=0,
                    help="only time --steps training steps (forward, loss, backward, gradient) "
                         "of the learned damping's MLP on this many synthetic sample rows")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        return 2

    import torch

    from paper_1610_07522_amd import inputs, sky

    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")   # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps(dict(copy_bytes=4 << 28, copies=3)), flush=True)
        return 0
    if args.mlp_rows > 0:
        if not torch.cuda.is_available():
            print("bench.py needs a ROCm GPU", file=sys.stderr)
            return 1
        return bench_mlp(args)
    if args.workload == "learned_protocol":
        if not torch.cuda.is_available():
            print("bench.py needs a ROCm GPU", file=sys.stderr)
            return 1
        return bench_learned_protocol(args)
    if args.to_residual > 0:
        if not torch.cuda.is_available():
            print("bench.py needs a ROCm GPU", file=sys.stderr)
            return 1
        return bench_to_residual(args)
    if args.workload == "batch64":
        if not torch.cuda.is_available():
            print("bench.py needs a ROCm GPU", file=sys.stderr)
            return 1
        return bench_batch(args)
    w = workload_of(args)
    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        return 1
    dev = torch.device("cuda:0")
    log(f"workload {w.name}: {w.n}^3, {w.n_neutrons} n + {w.n_protons} p "
        f"(+{w.extra_n} + {w.extra_p} extra states); generating inputs")
    t0 = time.perf_counter()
    raw_n, raw_p = inputs.raw_states(w)
    dn = torch.from_numpy(raw_n).to(dev)
    dp = torch.from_numpy(raw_p).to(dev)
    del raw_n, raw_p
    log(f"inputs on device in {time.perf_counter() - t0:.1f} s")

    def run(precision: int):
        box = sky.Box(sky.desc_from_workload(w, precision=precision, **form_kwargs(args)),
                      device=dev)
        t0 = time.perf_counter()
        box.init_box(dn, dp)
        torch.cuda.synchronize()
        tag = "mixed" if precision else "fp64"
        log(f"[{tag}] init (Loewdin, densities, mean field) {time.perf_counter() - t0:.1f} s")
        tuning = None
        if args.tune_cache != "off":
            t0 = time.perf_counter()
            tuning = box.autotune(args.tune_cache)
            log(f"[{tag}] launch shapes {tuning} ({time.perf_counter() - t0:.1f} s)")
            box.init_box(dn, dp)   # the tuner overwrote h psi and the subspace matrices
        for i in range(args.warmup):
            rep = box.iterate(1)
            log(f"[{tag}] warmup {i + 1}/{args.warmup}: residual {rep['residual']:.4e} "
                f"E {rep['energy']:.6f}")
        box.set_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = [box.iterate(1) for _ in range(args.steps)]
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        timing = box.timing()
        box.set_timing(False)
        box.close()
        del box
        torch.cuda.empty_cache()
        log(f"[{tag}] timed {args.steps} steps in {elapsed:.3f} s; last residual "
            f"{reps[-1]['residual']:.4e} E/A {reps[-1]['energy_per_a']:.6f}")
        return elapsed, timing, reps, tuning

    mixed = args.precision == "mixed"
    elapsed, timing, reps, tuning = run(sky.SKY_MIXED if mixed else sky.SKY_FP64)
    phases = {k: round((v["ms_n"] + v["ms_p"]) / args.steps, 3) for k, v in timing.items()}
    out = dict(
        metric="damped-gradient iterations/s, 48^3 box, 2000 nucleons",
        value=args.steps / elapsed, unit="iter/s", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=1e3 * elapsed / args.steps, higher_is_better=True,
        scaling="weak", vs_baseline=None,
        dtype=("mixed: c64 states, f32 FFT/h*psi, fp16x2-split MFMA GEMMs with f32->f64 "
               "accumulation, f64 subspace solve and sums") if mixed else "f64",
        data="synthetic",
        config=dict(workload=(f"{w.name}: {w.n}^3 grid, dx {w.dx} fm, {w.n_neutrons} n + "
                              f"{w.n_protons} p, rod-perturbed plane waves, SLy4"),
                    grid=w.n, nucleons=w.n_states, precision=args.precision,
                    **form_config(args, w)),
        roofline=roofline(timing, w, mixed),
        h_phase_hbm=h_phase_hbm(timing, w, mixed),
        hbm_phases=hbm_phases(timing, w, mixed),
        phases_ms_per_iter=phases,
        residual=reps[-1]["residual"], energy_per_a=reps[-1]["energy_per_a"],
        eigensolver=dict(iters_per_step=[r["eig_iters"] for r in reps],
                         jacobi_fallbacks=sum(r["eig_fallbacks"] for r in reps)),
        launch_shapes=tuning,
    )
    if mixed and not args.no_fp64_compare:
        e64, t64, r64, _ = run(sky.SKY_FP64)
        out["fp64_form"] = dict(value=args.steps / e64, ms_per_step=1e3 * e64 / args.steps,
                                speedup_mixed=(args.steps / elapsed) / (args.steps / e64),
                                phases_ms_per_iter={k: round((v["ms_n"] + v["ms_p"]) / args.steps, 3)
                                                    for k, v in t64.items()},
                                energy_per_a=r64[-1]["energy_per_a"])
    out["hbm_copy"] = copy_bandwidth(dev)
    del dn, dp
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(w)
        log("timing the CPU oracle in full on the 16^3 box")
        out["cpu_baseline"]["config_fermi16"] = oracle_config0()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
