#!/usr/bin/env python3
"""Throughput of the QTB-PIMD integrator step on one MI355X.

--workload batched-64 instead times the 64-replica sweep (3x3x3 .. 10x10x10
cells, 20 .. 1000 K, gamma 0.5 .. 20 /ps, P in {1, 4, 8}) stepping together.

Workload (default): MgO-like rock salt, 8x8x8 conventional cells (4096 atoms)
x P = 8 beads, QTB-PIMD at 50 K with the bead-modified spectrum kappa_P,
gamma = 1/ps, dt = 1 fs, 512-tap FIR blocked over K = 64 steps on BF16x3
matrix cores, FP32 forces with FP64 state.  A step is one pass of the whole
hot path: white noise + FIR (once per K steps), fused B/NM/A/O/A update,
neighbour-list check, pair forces with the closing kick.

Prints one JSON line: atom-bead-steps/s, the roofline of the dominant kernel
(pair forces, ALU bound) and of the FIR (HBM bytes), and the oracle timed on
the host cores on a bounded sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic work of one unique pair within r_cut, counted from the closed
# forms of the Buckingham (shifted-force) and damped-shifted-force Coulomb
# terms, each of rsqrt, exp, exp counted as one flop: 50 flops, or 47 VALU
# lane-slots with FMA fused and the transcendentals (rsqrt, the Buckingham
# and Gaussian exponentials) at four slots each, quarter rate.  Lane-slot
# peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (no packed FP32: the build
# disables it).
FLOPS_PER_PAIR = 50
SLOTS_PER_PAIR = 47
PEAK_LANE_SLOTS = 256 * 4 * 16 * 2.4e9
# Algorithmic HBM bytes of the FIR per dof-step: one white-noise value read and
# one coloured-noise value written, FP32 each.
FIR_BYTES_PER_DOF_STEP = 8
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0


# Sources whose change makes a stored HBM-traffic record of the pair kernel stale.
FORCE_SOURCES = ("paper_1905_02521_amd/csrc/forces.hip", "paper_1905_02521_amd/csrc/qtb_internal.h",
                 "paper_1905_02521_amd/csrc/force_epilogue.h", "paper_1905_02521_amd/csrc/ring_step.h")
PROFILES = os.path.join(ROOT, "profiles")


def source_hash(paths=FORCE_SOURCES):
    import hashlib
    h = hashlib.sha256()
    for rel in paths:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def stored_traffic(kernel_prefix="k_force_pair"):
    """HBM bytes per launch of the pair kernel from the committed counter
    summary (profiles/*traffic*.md, line 'traffic-record: {json}'), or None
    when no record exists or the kernel source changed since it was taken."""
    if not os.path.isdir(PROFILES):
        return None
    cur = source_hash()
    for fn in sorted(os.listdir(PROFILES)):
        if "traffic" not in fn:
            continue
        with open(os.path.join(PROFILES, fn)) as f:
            for line in f:
                if line.startswith("traffic-record:"):
                    rec = json.loads(line.split(":", 1)[1])
                    if rec.get("kernel", "").startswith(kernel_prefix) and rec.get("source") == cur:
                        return rec
    return None


def _short_name(name):
    n = name.replace("qtb::(anonymous namespace)::", "")
    if n.startswith("void "):
        n = n[5:]
    return n.split("(")[0]


def rocprof_summary(dirs):
    """Markdown summary of rocprofv3 CSV output: kernel stats of a trace run,
    or per-kernel mean counter values of --pmc runs.  With a FETCH_SIZE and a
    WRITE_SIZE run that include the bench's 256 MiB copy (--copy-calibration),
    the counters are scaled so the copy reads and writes exactly 256 MiB, and a
    traffic record of the pair kernel is printed."""
    import csv
    import collections
    out = []
    counters = collections.defaultdict(list)
    for d in dirs:
        stats = os.path.join(d, "run_kernel_stats.csv")
        if os.path.exists(stats):
            # medians from the per-dispatch trace (the average includes the rare
            # long launches, e.g. steps that rebuild neighbour lists)
            med = {}
            trace = os.path.join(d, "run_kernel_trace.csv")
            if os.path.exists(trace):
                durs = collections.defaultdict(list)
                for r in csv.DictReader(open(trace)):
                    durs[r["Kernel_Name"]].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
                med = {k: sorted(v)[len(v) // 2] for k, v in durs.items()}
            out.append(f"| kernel | calls | avg us | median us | min us | max us | % of GPU time |")
            out.append("|---|---|---|---|---|---|---|")
            for r in csv.DictReader(open(stats)):
                m = med.get(r["Name"])
                ms = f"{m / 1e3:.2f}" if m is not None else ""
                out.append(f"| {_short_name(r['Name'])} | {r['Calls']} | "
                           f"{float(r['AverageNs']) / 1e3:.2f} | {ms} | {float(r['MinNs']) / 1e3:.2f} | "
                           f"{float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")
        cc = os.path.join(d, "run_counter_collection.csv")
        if os.path.exists(cc):
            per = collections.defaultdict(float)
            for r in csv.DictReader(open(cc)):
                per[(r["Dispatch_Id"], r["Kernel_Name"], r["Counter_Name"])] += float(r["Counter_Value"])
            for (disp, k, c), v in per.items():
                counters[(_short_name(k), c)].append(v)
    if counters:
        copy_bytes = 256 * 2 ** 20
        scale = {}
        for c in ("FETCH_SIZE", "WRITE_SIZE"):
            v = counters.get(("__amd_rocclr_copyBuffer", c))
            if v:
                scale[c] = copy_bytes / (max(v) * 1024.0)
        out.append("")
        out.append("| kernel | counter | dispatches | mean per dispatch | scaled bytes |")
        out.append("|---|---|---|---|---|")
        for (k, c), v in sorted(counters.items()):
            m = sum(v) / len(v)
            sb = f"{m * 1024 * scale[c]:.4g}" if c in scale else ""
            out.append(f"| {k} | {c} | {len(v)} | {m:.6g} | {sb} |")
        # VALU activity of the pair kernel (rocprof's VALUBusy / VALUUtilization;
        # GRBM_GUI_ACTIVE is summed over the 8 XCDs, so one XCD's busy cycles
        # are the sum / 8)
        fk = [k for (k, c) in counters if k.startswith("k_force_pair")]
        have = {c for (k, c) in counters if fk and k == fk[0]}
        if fk and {"SQ_ACTIVE_INST_VALU", "GRBM_GUI_ACTIVE", "SQ_THREAD_CYCLES_VALU"} <= have:
            k = fk[0]
            mean = lambda c: sum(counters[(k, c)]) / len(counters[(k, c)])
            busy = 100.0 * mean("SQ_ACTIVE_INST_VALU") / 256 / (mean("GRBM_GUI_ACTIVE") / 8)
            util = 100.0 * mean("SQ_THREAD_CYCLES_VALU") / (mean("SQ_ACTIVE_INST_VALU") * 64)
            out.append("")
            out.append(f"{k}: VALUBusy {busy:.1f} % (VALU-active cycles per CU over one XCD's busy "
                       f"cycles), VALUUtilization {util:.1f} % (active lanes per VALU cycle)")
        if scale:
            out.append("")
            out.append("copy calibration (bytes per KiB-unit of the counter): " +
                       ", ".join(f"{c} x{s * 1024:.1f} (factor {s:.4f})" for c, s in scale.items()))
            fk = [k for (k, c) in counters if k.startswith("k_force_pair")]
            if fk and all(c in scale for c in ("FETCH_SIZE", "WRITE_SIZE")):
                k = fk[0]
                rd = sum(counters[(k, "FETCH_SIZE")]) / len(counters[(k, "FETCH_SIZE")])
                wr = sum(counters[(k, "WRITE_SIZE")]) / len(counters[(k, "WRITE_SIZE")])
                rec = {"kernel": k, "source": source_hash(),
                       "fetch_bytes": rd * 1024 * scale["FETCH_SIZE"],
                       "write_bytes": wr * 1024 * scale["WRITE_SIZE"]}
                rec["bytes"] = rec["fetch_bytes"] + rec["write_bytes"]
                out.append("")
                out.append("traffic-record: " + json.dumps(rec))
    return "\n".join(out)


def unique_pairs(beads, box, r_cut):
    """Number of distinct pairs (with periodic images) within r_cut, summed
    over beads: the algorithmic unit of the force kernel."""
    from scipy.spatial import cKDTree
    n = 0
    for b in range(beads.shape[0]):
        x = np.mod(beads[b].T, box)
        if np.min(box) > 2 * r_cut:
            t = cKDTree(x, boxsize=box)
            n += len(t.query_pairs(r_cut, output_type="ndarray"))
        else:
            # small box: every image within r_cut counts (i<j, plus i=j images once)
            m = [int(np.ceil(r_cut / L)) for L in box]
            shifts = np.array([(i, j, k) for i in range(-m[0], m[0] + 1)
                               for j in range(-m[1], m[1] + 1)
                               for k in range(-m[2], m[2] + 1)]) * box
            d = x[:, None, :] - x[None, :, :]
            d -= box * np.rint(d / box)
            cnt = 0
            for sh in shifts:
                r2 = np.sum((d + sh) ** 2, axis=-1)
                cnt += np.count_nonzero(r2 < r_cut * r_cut) - (x.shape[0] if not sh.any() else 0)
            n += cnt // 2
    return n


def host_cpu():
    """The host the oracle ran on: logical CPUs, those this process may use,
    and the CPU model."""
    model = ""
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
    except (AttributeError, OSError):
        usable = os.cpu_count() or 1
    return {"nproc": os.cpu_count(), "usable_cpus": usable, "cpu_model": model}


def cpu_baseline(w, beads, sp, box, pot, budget_s=15.0):
    """The oracle (plain FP64 C, OpenMP over atoms) on the same workload,
    bounded to about budget_s seconds of stepping."""
    from oracle import oracle as orc
    from paper_1905_02521_amd import workloads as W
    threads = min(host_cpu()["usable_cpus"], 16)
    U = orc.make_units(**W.METAL_UNITS)
    opot = orc.make_pot(0, pot.mass, pot.charge, pot.buck_A, pot.buck_rho, pot.buck_C,
                        pot.dsf_alpha, pot.r_cut, pot.skin)
    N, P = beads.shape[2], beads.shape[0]
    sim = orc.Sim(opot, U, N, P, 3, box, sp, w.T, w.gamma, w.dt, w.seed, w.stream, w.noise,
                  w.two_nf, beads, n_threads=threads)
    sim.run(1)  # first step outside the clock
    n, t = 0, 0.0
    while t < budget_s and n < 10000:
        k = 1 if n == 0 else max(1, int(n * (budget_s - t) / max(t, 1e-9) / 2))
        k = min(k, 200)
        t0 = time.perf_counter()
        sim.run(k)
        t += time.perf_counter() - t0
        n += k
    return {"value": N * P * n / t, "unit": "atom-bead-steps/s", "cores": threads,
            "kind": "oracle", "_ab": N * P * n, "_t": t, **host_cpu(),
            "sample": f"{n} steps of the same workload ({N} atoms x {P} beads), "
                      f"{t:.1f} s, FP64, {threads} OpenMP threads"}


def surrogate_bench(a):
    """The learned surrogate on the 20x20x20-cell crystal x P = 4 (QTB-PIMD,
    300 K): trained on the GPU on frames of the method's own QTB (P = 1 at
    16 temperatures from 50 to 1000 K) and QTB-PIMD (P = 4 at 50 to 300 K)
    runs of the 4x4x4 crystal, labelled by the pair potential, by mini-batch
    Adam; held-out force and energy errors; then timed against the pair
    potential on the production workload, with the pair potential's check of
    the force error every 64 steps."""
    import torch
    from paper_1905_02521_amd import qtb, surrogate, workloads as W
    pot = W.mgo_potential(skin=a.skin)
    U = dict(W.METAL_UNITS)
    t_gen = time.perf_counter()
    # QTB at 16 temperatures 50 * 20^(j / 15) K (50 to 1000 K), and QTB-PIMD
    # with P = 4 at 50, 100 and 300 K: the production run's bead configurations
    conds = ([(round(50.0 * 20.0 ** (j / 15.0), 1), 1) for j in range(16)] +
             [(50.0, 4), (100.0, 4), (300.0, 4)])
    frames, forces, energies, sp, box, tags = surrogate.qtb_frames(pot, conds, n_frames=a.ml_samples,
                                                                   every=40, warm=2000)
    t_gen = time.perf_counter() - t_gen
    print(f"surrogate: {len(frames)} frames in {t_gen:.1f} s", file=sys.stderr, flush=True)
    perm = np.random.default_rng(0).permutation(len(frames))
    n_test = len(frames) // 5
    te, tr = perm[:n_test], perm[n_test:]
    model = qtb.Model(6.0, 0.5)
    model.init_params(1)
    n_train = a.ml_steps
    torch.cuda.synchronize()
    t_train = time.perf_counter()
    losses = surrogate.train(model, pot, frames[tr], forces[tr], energies[tr], sp, box,
                             steps=n_train, batch=256)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t_train
    print(f"surrogate: {n_train} training steps in {t_train:.1f} s", file=sys.stderr, flush=True)
    test_rmse, test_rel, test_e = surrogate.errors(model, pot, frames[te], forces[te],
                                                   energies[te], sp, box)
    by_cond = {}
    for T, P in conds:
        sel = np.array([k for k in te if tags[k] == (T, P)])
        if len(sel):
            r_, rel_, e_ = surrogate.errors(model, pot, frames[sel], forces[sel], energies[sel],
                                            sp, box)
            by_cond[f"T{T:.0f}-P{P}"] = {"force_rmse_eV_A": r_, "force_rel_rmse": rel_,
                                         "energy_rmse_eV_per_atom": e_, "frames": int(len(sel))}
    n_at = len(sp)
    # production workload
    n, P = 20, 4
    pos, sp2, box2 = W.rocksalt(n)
    rep = qtb.Replica(pos=W.beads_from(W.displaced(pos, 0.0421, 4), P), species=sp2, T=300.0,
                      gamma=1e-3, dt=1.0, noise=2, box=tuple(box2), seed=4)
    ctx = qtb.Context(qtb.pair_potential_dict(pot), [rep], U, prec=qtb.PREC_FP32,
                      fir=qtb.FIR_BF16X3, ml_r_cut=6.0)
    ctx.build_filter(0, 2, 512)
    ab = n ** 3 * 8 * P
    ctx.step(128)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(512)
    torch.cuda.synchronize()
    plain_s = (time.perf_counter() - t0) / 512
    ctx.ml_attach(model, check_every=64)
    ctx.step(128)
    ctx.ml_check(0)
    torch.cuda.synchronize()
    steps = 256
    t0 = time.perf_counter()
    ctx.step(steps)
    torch.cuda.synchronize()
    ml_s = (time.perf_counter() - t0) / steps
    rmse, rel, n_chk = ctx.ml_check(0)
    ctx.profile(True)
    ctx.step(16)
    prof = ctx.profile_read()
    ctx.profile(False)
    ctx.close()
    out = {
        "metric": "atom-bead-steps/s per GPU (surrogate forces + QTB noise + update)",
        "value": ab / ml_s, "unit": "atom-bead-steps/s", "n_gpus": 1, "steps": steps,
        "ms_per_step": ml_s * 1e3, "higher_is_better": True, "dtype": "f32 (bf16 weights)",
        "data": "synthetic (seeded rock-salt crystal; training frames from the method's own "
                "QTB and QTB-PIMD runs of the pair potential, labelled by it)",
        "config": {"workload": "surrogate-20x20x20-P4", "atoms": n ** 3 * 8, "beads": P,
                   "atom_beads_per_step": ab, "T_K": 300.0, "noise": "QTB-PIMD kappa_P",
                   "r_ml_A": 6.0, "network": "96-64-64-1 silu per species"},
        "plain": {"value": ab / plain_s, "ms_per_step": plain_s * 1e3},
        "surrogate_over_plain": plain_s / ml_s,
        "accuracy": {"test_force_rmse_eV_A": test_rmse, "test_force_rel_rmse": test_rel,
                     "test_energy_rmse_eV_per_atom": test_e, "test_frames": int(n_test),
                     "by_condition": by_cond,
                     "run_check_force_rmse_eV_A": rmse, "run_check_rel_rmse": rel,
                     "run_checks": n_chk},
        "training": {"frames": int(len(tr)), "atoms_per_frame": n_at,
                     "frame_sources": "QTB P=1 at 16 T from 50 to 1000 K, QTB-PIMD P=4 beads at 50-300 K",
                     "frame_generation_s": t_gen, "adam_steps": n_train, "batch_frames": 256,
                     "first_loss": float(losses[0]), "last_loss": float(losses[-1]),
                     "ms_per_step": t_train / n_train * 1e3},
        "winner": ("pair potential" if plain_s < ml_s else "surrogate") +
                  " (faster per step; the surrogate approximates the pair potential, "
                  "which is also its reference)",
        "phases_ms_per_step": {k: v[0] / 16 for k, v in prof.items()},
    }
    print(json.dumps(out))


def pimd_compare_bench(a):
    """QTB (P = 1, theta noise), QTB-PIMD (kappa_P noise) and classical PIMD
    (white noise) on the 4x4x4 MgO crystal at 50 K.

    Cost: one replica of each of QTB, QTB-PIMD P = 8 and PIMD P = 32 at
    gamma = 1/ps, time per step, beside the paper's statement that QTB needs
    about a twentieth of the PIMD computation time (its hardware and workload
    are not stated).

    Convergence in P (Sec. 2.3, Fig. 8: QTB-PIMD converges with far fewer
    beads): one batched context of three replicas per condition, PIMD at
    P = 32 and 64, QTB-PIMD at P = 4, 8, 16 (gamma = 1/ps) and at P = 8 with
    gamma = 2, 0.5, 0.25 /ps and with a 2048-tap filter, QTB at gamma = 1 and
    0.25 /ps; 20 000 steps of equilibration, then a.blocks blocks of 5000
    steps.  Per condition the block means (eV/atom) of the potential energy
    (free of any kinetic estimator), the centroid-virial and primitive
    energies and the pressure, and PIMD's P -> infinity limit from P = 32
    and 64 with the 1/P^2 law of the primitive discretisation."""
    import torch
    from paper_1905_02521_amd import qtb, workloads as W
    pot = W.mgo_potential(skin=1.0)
    U = dict(W.METAL_UNITS)
    pos, sp, box = W.rocksalt(4)
    base = W.displaced(pos, 0.0421, 2)
    N = len(sp)
    out_runs = {}
    for name, P, noise in (("qtb", 1, 1), ("qtb-pimd", 8, 2), ("pimd", 32, 0)):
        rep = qtb.Replica(pos=W.beads_from(base, P), species=sp, T=50.0, gamma=1e-3, dt=1.0,
                          noise=noise, box=tuple(box), seed=2)
        ctx = qtb.Context(qtb.pair_potential_dict(pot), [rep], U, prec=qtb.PREC_FP32,
                          fir=qtb.FIR_BF16X3, obs_every=8, max_two_nf=512)
        if noise:
            ctx.build_filter(0, noise, 512)
        ctx.step(2000)
        ctx.observables(0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.step(a.steps * 4)
        ctx.observables(0)
        dt = (time.perf_counter() - t0) / (a.steps * 4)
        ctx.close()
        out_runs[name] = {"beads": P, "ms_per_step": dt * 1e3, "atom_bead_steps_per_s": N * P / dt}
    conds = [("pimd-P32", 32, 0, 1e-3, 512), ("pimd-P64", 64, 0, 1e-3, 512),
             ("qtbpimd-P4", 4, 2, 1e-3, 512), ("qtbpimd-P8", 8, 2, 1e-3, 512),
             ("qtbpimd-P16", 16, 2, 1e-3, 512), ("qtbpimd-P8-gamma2", 8, 2, 2e-3, 512),
             ("qtbpimd-P8-gamma0.5", 8, 2, 5e-4, 512), ("qtbpimd-P8-gamma0.25", 8, 2, 2.5e-4, 1024),
             ("qtbpimd-P8-2Nf2048", 8, 2, 1e-3, 2048), ("qtb", 1, 1, 1e-3, 512),
             ("qtb-gamma0.25", 1, 1, 2.5e-4, 1024)]
    n_r = 3
    reps, keys = [], []
    for name, P, noise, g, nf in conds:
        for k in range(n_r):
            b0 = W.displaced(pos, 0.02, 10 + k)
            beads = (b0[None] if P == 1 else
                     np.stack([W.displaced(b0, 0.005, 100 + 10 * k + b) for b in range(P)]))
            reps.append(qtb.Replica(pos=beads, species=sp, T=50.0, gamma=g, dt=1.0, noise=noise,
                                    box=tuple(box), seed=300 + len(reps), stream=len(reps)))
            keys.append((name, noise, nf))
    ctx = qtb.Context(qtb.pair_potential_dict(pot), reps, U, prec=qtb.PREC_FP32,
                      fir=qtb.FIR_BF16X3, obs_every=8, max_two_nf=2048)
    for r, (_, noise, nf) in enumerate(keys):
        if noise:
            ctx.build_filter(r, noise, nf)
    ctx.step(20_000)
    for r in range(len(keys)):
        ctx.observables(r)
    fields = ("potential", "e_virial", "e_primitive", "pressure")
    blocks = {c[0]: {f: [] for f in fields} for c in conds}
    for _ in range(a.blocks):
        ctx.step(5000)
        acc = {c[0]: {f: [] for f in fields} for c in conds}
        for r, (name, _, _) in enumerate(keys):
            o = ctx.observables(r)
            for f in fields:
                acc[name][f].append(o[f] / (1 if f == "pressure" else N))
        for c in conds:
            for f in fields:
                blocks[c[0]][f].append(float(np.mean(acc[c[0]][f])))
    ctx.close()
    conv = {}
    for c in conds:
        conv[c[0]] = {f: [float(np.mean(v)), float(np.std(v, ddof=1) / math.sqrt(len(v)))]
                      for f, v in blocks[c[0]].items()}
    lim = {}
    for f in fields:   # X(P) = X_inf + c / P^2 through P = 32 and 64
        (m32, s32), (m64, s64) = conv["pimd-P32"][f], conv["pimd-P64"][f]
        lim[f] = [m64 + (m64 - m32) / 3.0, math.hypot(4.0 * s64, s32) / 3.0]
    conv["pimd-P-infinity"] = lim
    out = {
        "metric": "QTB vs QTB-PIMD vs PIMD: time per step and the energies' convergence in P",
        "unit": "ms/step; eV/atom and eV/A^3 (mean, standard error of block means)",
        "n_gpus": 1, "higher_is_better": False, "dtype": "f32",
        "data": "synthetic (seeded rock-salt crystal, numpy PCG64 displacements)",
        "config": {"workload": "mgo-4x4x4-50K-qtb-vs-pimd", "atoms": N, "T_K": 50.0,
                   "replicas_per_condition": n_r, "equilibration_steps": 20_000,
                   "blocks": a.blocks, "block_steps": 5000},
        "runs": out_runs,
        "pimd_over_qtb_time": out_runs["pimd"]["ms_per_step"] / out_runs["qtb"]["ms_per_step"],
        "pimd_over_qtbpimd_time": (out_runs["pimd"]["ms_per_step"] /
                                   out_runs["qtb-pimd"]["ms_per_step"]),
        "convergence": conv,
        "paper": "QTB about 20x cheaper than PIMD (abstract; hardware and workload not stated)",
    }
    print(json.dumps(out))


def vdos_bench(a):
    """Velocity density of states on the 8x8x8 MgO crystal (4096 atoms, QTB,
    P = 1, 50 K, gamma = 1/ps, every step sampled, segments of 1024 samples):
    the step time with sampling alone and with the velocity recorder attached
    (the recorder's cost inside the step kernels plus one transform per
    segment), and the transform by itself on a seeded trace of the same shape
    (12288 dofs x 1024 samples, FP64): its time per segment and its rate
    against HBM, counting one read of the segment as the algorithmic traffic."""
    import torch
    from paper_1905_02521_amd import qtb, workloads as W
    pot = W.mgo_potential(skin=0.4)
    pos, sp, box = W.rocksalt(8)
    base = W.displaced(pos, 0.0421, 2)
    N, seg, n_seg = len(sp), 1024, 8
    n_dof = 3 * N
    # one context (one force-kernel decomposition): sampling alone, then with
    # the recorder attached, then sampling alone again
    rep = qtb.Replica(pos=W.beads_from(base, 1), species=sp, T=50.0, gamma=1e-3, dt=1.0,
                      noise=1, box=tuple(box), seed=2)
    ctx = qtb.Context(qtb.pair_potential_dict(pot), [rep], W.METAL_UNITS, prec=qtb.PREC_FP32,
                      fir=qtb.FIR_BF16X3, obs_every=1, max_two_nf=512)
    ctx.build_filter(0, 1, 512)
    ctx.step(a.warmup)
    times = {"sampling": [], "recorder": []}
    for name in ("sampling", "recorder", "sampling"):
        if name == "recorder":
            ctx.vdos_attach(0, seg)
        ctx.observables(0)
        t0 = time.perf_counter()
        ctx.step(seg * n_seg)
        if name == "recorder":
            assert ctx.vdos_read(0)[1] == n_seg
        ctx.observables(0)
        times[name].append((time.perf_counter() - t0) / (seg * n_seg))
        if name == "recorder":
            ctx.vdos_detach(0)
    ctx.close()
    times = {k: sum(v) / len(v) for k, v in times.items()}
    # the transform alone, timed with events on the stream it runs on, on
    # the recorder's layout (one row of dofs per sample) and on contiguous
    # series per dof
    g = torch.Generator(device="cpu").manual_seed(7)
    wts = torch.full((n_dof,), 24.3, dtype=torch.float64, device="cuda")
    t_seg = {}
    for layout in ("dof_major", "sample_major"):
        shape = (n_dof, seg * n_seg) if layout == "dof_major" else (seg * n_seg, n_dof)
        v = torch.randn(shape, generator=g, dtype=torch.float64).cuda()
        for _ in range(3):
            qtb.vdos_spectrum(v, wts, seg, dof_major=layout == "dof_major")
        torch.cuda.synchronize()
        reps = 20
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            qtb.vdos_spectrum(v, wts, seg, dof_major=layout == "dof_major")
        e1.record()
        torch.cuda.synchronize()
        t_seg[layout] = e0.elapsed_time(e1) * 1e-3 / (reps * n_seg)
        del v
    bytes_seg = 8.0 * seg * n_dof
    out = {
        "metric": "velocity spectrum: recorder overhead per step, transform rate",
        "unit": "ms/step; us/segment; GB/s",
        "n_gpus": 1, "higher_is_better": True, "dtype": "f64",
        "data": "synthetic (seeded rock-salt crystal; seeded Gaussian trace)",
        "config": {"workload": "mgo-8x8x8-qtb-50K-vdos", "atoms": N, "dofs": n_dof,
                   "segment_samples": seg, "segments": n_seg},
        "ms_per_step_sampling": times["sampling"] * 1e3,
        "ms_per_step_recorder": times["recorder"] * 1e3,
        "recorder_overhead": times["recorder"] / times["sampling"] - 1.0,
        "transform_us_per_segment": t_seg["sample_major"] * 1e6,
        "transform_us_per_segment_dof_major": t_seg["dof_major"] * 1e6,
        "transform": {"bound": "hbm", "achieved": bytes_seg / t_seg["sample_major"] / 1e9,
                      "peak": 8000.0, "unit": "GB/s",
                      "frac": bytes_seg / t_seg["sample_major"] / 8e12,
                      "bytes_per_segment": bytes_seg},
    }
    print(json.dumps(out))


def sweep_heat_capacity(works, inputs, pot, a):
    """Heat capacity per replica of the batched sweep: every replica beside a
    twin at T (1 + 0.05) with the same cells, beads, friction, filter length,
    start and white-noise stream (correlated sampling: the twins differ only
    in the filter's temperature, so most of the noise cancels in their
    energy difference), production precision.  Equilibration of 10/gamma of
    the weakest friction, then a.hc_blocks x 2/gamma steps sampled every 8
    and read out in windows of about 1/(8 gamma) (whole noise blocks).  C = (E(T') - E(T)) / (T' - T)
    per atom in units of 3 k_B, with the standard error of the windows'
    paired differences by blocking (Flyvbjerg-Petersen), from three
    energies: the eq. 5 primitive energy and the centroid-virial energy
    (both with measured momenta, so both carry the friction tail of the
    Langevin dynamics; the primitive one with the internal ring-polymer
    modes' share, which shrinks as T, and with it omega_P, grows), and twice
    the bead-averaged potential energy (no momenta; equal to the total
    energy for harmonic modes)."""
    from paper_1905_02521_amd import qtb, workloads as W
    from paper_1905_02521_amd.stats import mean_and_error
    reps = []
    for k, w in enumerate(works):
        beads, sp, box = inputs[k]
        for T in (w.T, 1.05 * w.T):
            reps.append(qtb.Replica(pos=beads, species=sp, T=T, gamma=w.gamma, dt=w.dt,
                                    noise=w.noise, box=tuple(box), seed=w.seed + 1000,
                                    stream=w.stream))
    ctx = qtb.Context(qtb.pair_potential_dict(pot), reps, W.METAL_UNITS, prec=qtb.PREC_FP32,
                      fir=qtb.FIR_BF16X3, obs_every=8,
                      max_two_nf=max(max(w.two_nf, 2) for w in works))
    for k, w in enumerate(works):
        if w.noise:
            for twin in (0, 1):
                ctx.build_filter(2 * k + twin, w.noise, w.two_nf)
    tau = 1.0 / min(w.gamma * w.dt for w in works)
    warm, block = int(10 * tau), int(2 * tau)
    window = 64 * max(1, round(block / 16 / 64))   # whole noise blocks
    ctx.step(warm)
    for r in range(len(reps)):
        ctx.observables(r)
    fields = (("C_prim", "e_primitive", 1.0), ("C_vir", "e_virial", 1.0),
              ("C_2V", "potential", 2.0))
    blocks = [{f: [] for _, f, _ in fields} for _ in reps]
    for q in range(a.hc_blocks):
        for _ in range(block // window):
            ctx.step(window)
            for r in range(len(reps)):
                o = ctx.observables(r)
                for _, f, _ in fields:
                    blocks[r][f].append(o[f])
        print(f"heat capacity: {q + 1}/{a.hc_blocks} x {block} steps", file=sys.stderr,
              flush=True)
    ctx.close()
    kB = W.METAL_UNITS["kB"]
    out = []
    for k, w in enumerate(works):
        n_at = inputs[k][0].shape[2]
        scale = 1.0 / (0.05 * w.T * 3 * kB * n_at)
        e = {"T_K": round(w.T, 2), "beads": w.P, "gamma_per_ps": round(w.gamma * 1e3, 3),
             "atoms": int(n_at)}
        for name, f, mult in fields:
            d = mult * scale * (np.array(blocks[2 * k + 1][f]) - np.array(blocks[2 * k][f]))
            m, se = mean_and_error(d)
            e[name] = [m, se]
        out.append(e)
    return {"twin_dT": "0.05 T", "equilibration_steps": warm,
            "sampled_steps": a.hc_blocks * (block // window) * window, "window_steps": window,
            "error": "blocking (Flyvbjerg-Petersen) over the windows' paired differences",
            "units": "3 k_B per atom, [mean, standard error]",
            "replicas": out}


def fir_modes_bench(a):
    """The default workload (MgO 8x8x8 x P = 8, 50 K, kappa_P, 2Nf = 512,
    K = 64, FP32 forces) with each FIR arithmetic: wall time per step over
    whole noise blocks, and the FIR and white-noise GPU time per block from
    the dispatch stamps of four further blocks.  The FIR's algorithmic bytes
    are 8 per noise value (one new white-noise value read, one coloured value
    written: 98 304 columns x 64 steps per block).  The FP64 FIR runs with
    FP64 forces and state (the library pairs them)."""
    from paper_1905_02521_amd import qtb, workloads as W
    w = W.workload("mgo-8x8x8-qtbpimd-P8-50K")
    beads, sp, box = W.crystal_inputs(w)
    n_dof = beads.size
    K = 64
    steps = max(K, (a.steps // K) * K)
    res = {}
    for name, fir in (("fp64", qtb.FIR_FP64), ("fp32", qtb.FIR_FP32),
                      ("bf16x3", qtb.FIR_BF16X3), ("bf16", qtb.FIR_BF16)):
        rep = qtb.Replica(pos=beads, species=sp, T=w.T, gamma=w.gamma, dt=w.dt, noise=w.noise,
                          box=tuple(box), seed=w.seed, stream=w.stream)
        ctx = qtb.Context(qtb.pair_potential_dict(W.mgo_potential(skin=0.4)), [rep],
                          W.METAL_UNITS, prec=qtb.PREC_FP64 if name == "fp64" else qtb.PREC_FP32,
                          fir=fir, fir_block_K=K, max_two_nf=w.two_nf)
        ctx.build_filter(0, w.noise, w.two_nf)
        ctx.step(2 * K)
        ctx.get_state(0)   # synchronises
        t0 = time.perf_counter()
        ctx.step(steps)
        ctx.get_state(0)
        t = (time.perf_counter() - t0) / steps
        ctx.profile(True)
        ctx.step(4 * K)
        prof = ctx.profile_read()
        ctx.profile(False)
        ctx.close()
        fir_us = prof["fir"][0] / 4 * 1e3
        res[name] = {"ms_per_step": t * 1e3, "atom_bead_steps_per_s": n_dof / 3 / t,
                     "fir_us_per_block": fir_us,
                     "white_noise_us_per_block": prof["noise"][0] / 4 * 1e3,
                     "fir_GB_s": 8.0 * n_dof * K / (fir_us * 1e-6) / 1e9}
    out = {"metric": "atom-bead-steps/s per FIR arithmetic", "value": res["bf16x3"]["atom_bead_steps_per_s"],
           "unit": "atom-bead-steps/s", "n_gpus": 1, "steps": steps, "warmup": 2 * K,
           "ms_per_step": res["bf16x3"]["ms_per_step"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "bf16x3 noise, f32 forces",
           "data": "synthetic (seeded rock-salt crystal, numpy PCG64 displacements)",
           "config": {"workload": "mgo-8x8x8-qtbpimd-P8-50K", "fir_block_K": K,
                      "noise_columns": n_dof},
           "modes": res}
    print(json.dumps(out))


def npt_bench(a):
    """Constant pressure on the 8x8x8 MgO crystal (4096 atoms, FP32 forces,
    BF16x3 noise): wall time per step at constant volume and under a
    barostat at P0 = 0, where every step also samples K, the springs and the
    pair virial and runs the barostat update and its box commit (the lists
    follow the box by their scale factor and rebuild only when the skin runs
    out); GPU time per phase from the dispatch stamps of 256 further steps.
    Two cases: QTB (P = 1, 300 K, gamma = 1/ps) under cell rescaling
    (tau_p = 500 fs, beta_T = 1 A^3/eV), the headline, and QTB-PIMD (P = 8,
    50 K, kappa_P noise) under the Langevin piston (500 fs, 0.005 / fs).
    The oracle with the first case's barostat runs on the host cores."""
    from paper_1905_02521_amd import qtb, workloads as W
    pot = W.mgo_potential(skin=0.4)
    pos, sp, box = W.rocksalt(8)
    base = W.displaced(pos, 0.0421, 2)
    N = len(sp)
    T, gamma, dt, P0, tau_p, beta_T = 300.0, 1e-3, 1.0, 0.0, 500.0, 1.0

    def case(P, T_K, noise, enable):
        beads = (W.beads_from(base, 1) if P == 1 else
                 np.stack([W.displaced(base, 0.005, 300 + b) for b in range(P)]))
        rep = qtb.Replica(pos=beads, species=sp, T=T_K, gamma=gamma, dt=dt, noise=noise,
                          box=tuple(box), seed=2)
        ctx = qtb.Context(qtb.pair_potential_dict(pot), [rep], W.METAL_UNITS,
                          prec=qtb.PREC_FP32, fir=qtb.FIR_BF16X3, obs_every=64, max_two_nf=512)
        ctx.build_filter(0, noise, 512)
        ctx.step(a.warmup)
        t_step, phases = {}, {}
        for name in ("nvt", "npt"):
            if name == "npt":
                enable(ctx)
                ctx.step(a.warmup)
            ctx.observables(0)   # synchronises
            t0 = time.perf_counter()
            ctx.step(a.steps)
            ctx.observables(0)
            t_step[name] = (time.perf_counter() - t0) / a.steps
            ctx.profile(True)
            ctx.step(256)
            prof = ctx.profile_read()
            ctx.profile(False)
            phases[name] = {k: v[0] / 256 for k, v in prof.items() if v[1] > 0}
        box_end = ctx.box(0)
        ctx.close()
        return t_step, phases, box_end

    t_step, phases, box_end = case(1, T, 1, lambda c: c.barostat(0, P0, tau_p, beta_T))
    t_rp, ph_rp, box_rp = case(8, 50.0, 2, lambda c: c.piston(0, P0, tau_p, 0.005))
    out = {
        "metric": "atom-steps/s at constant pressure (forces+QTB noise+update+barostat)",
        "value": N / t_step["npt"], "unit": "atom-steps/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": t_step["npt"] * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded rock-salt crystal, numpy PCG64 displacements)",
        "config": {"workload": "mgo-8x8x8-qtb-300K-npt", "atoms": N, "P0_eV_A3": P0,
                   "tau_p_fs": tau_p, "beta_T_A3_eV": beta_T, "skin_A": 0.4},
        "ms_per_step_nvt": t_step["nvt"] * 1e3,
        "npt_cost": t_step["npt"] / t_step["nvt"] - 1.0,
        "phases_ms_per_step": {"nvt": phases["nvt"], "npt": phases["npt"]},
        "box_end_A": float(box_end[0]),
        "ring_polymer_piston": {
            "workload": "mgo-8x8x8-qtbpimd-P8-50K-piston", "beads": 8,
            "tau_p_fs": tau_p, "gamma_p_per_fs": 0.005,
            "ms_per_step_nvt": t_rp["nvt"] * 1e3, "ms_per_step_npt": t_rp["npt"] * 1e3,
            "npt_cost": t_rp["npt"] / t_rp["nvt"] - 1.0,
            "atom_bead_steps_per_s": N * 8 / t_rp["npt"],
            "phases_ms_per_step": ph_rp, "box_end_A": float(box_rp[0])},
    }
    if not a.no_cpu:
        from oracle import oracle as orc
        threads = min(os.cpu_count() or 1, 16)
        U = orc.make_units(**W.METAL_UNITS)
        opot = orc.make_pot(0, pot.mass, pot.charge, pot.buck_A, pot.buck_rho, pot.buck_C,
                            pot.dsf_alpha, pot.r_cut, pot.skin)
        sim = orc.Sim(opot, U, N, 1, 3, box, sp, T, gamma, dt, 2, 0, 1, 512,
                      W.beads_from(base, 1), n_threads=threads)
        sim.set_barostat(P0, tau_p, beta_T)
        sim.run(1)
        n, t = 0, 0.0
        while t < a.cpu_seconds and n < 10000:
            t0 = time.perf_counter()
            sim.run(20)
            t += time.perf_counter() - t0
            n += 20
        out["cpu_baseline"] = {"value": N * n / t, "unit": "atom-steps/s", "cores": threads,
                               "kind": "oracle",
                               "sample": f"{n} steps of the same workload with the barostat "
                                         f"({N} atoms), {t:.1f} s, FP64, {threads} OpenMP threads"}
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=640)
    ap.add_argument("--warmup", type=int, default=64)
    ap.add_argument("--workload", default="mgo-8x8x8-qtbpimd-P8-50K",
                    help="a named single workload, batched-64 (the T / gamma / P sweep) or "
                         "surrogate-20x20x20-P4 (the learned force surrogate) or qtb-vs-pimd "
                         "(QTB, QTB-PIMD and PIMD cost and energies on one crystal) or vdos "
                         "(the velocity spectrum's recorder and transform) or npt (the step "
                         "at constant pressure) or fir-modes (the default workload with each "
                         "FIR arithmetic)")
    ap.add_argument("--cells", type=int, default=0,
                    help="run a single crystal workload on n x n x n cells instead of its own size")
    ap.add_argument("--fir", default="bf16x3", choices=["fp32", "bf16x3", "bf16", "fp64"])
    ap.add_argument("--K", type=int, default=64)
    ap.add_argument("--noise-blocks", action="store_true",
                    help="make the coloured noise with the paper's block generator (eq. 9, "
                         "blocks of max two_nf steps) instead of the streaming FIR")
    ap.add_argument("--blocks", type=int, default=40,
                    help="qtb-vs-pimd: measured blocks of 5000 steps of the convergence sweep")
    ap.add_argument("--skin-full-T", type=float, default=600.0,
                    help="batched workloads: replicas at or above this temperature keep the full "
                         "skin, colder ones a thinner one, skin sqrt(T / this) (0: one skin)")
    ap.add_argument("--skin-min", type=float, default=0.8,
                    help="batched workloads: the thinnest per-replica skin (A)")
    ap.add_argument("--decomposition", default=None,
                    help="pin the pair-force decomposition instead of autotuning it: "
                         "waves per atom (1, 2 or 4), optionally ',half' for half bead groups")
    ap.add_argument("--hc-blocks", type=int, default=8,
                    help="batched workloads: blocks of 2/gamma for the heat capacity of every "
                         "replica (0: skip)")
    ap.add_argument("--ml-samples", type=int, default=7143,
                    help="surrogate workload: samples per training replica (19 replicas; the "
                         "three QTB-PIMD ones give 4 frames per sample: 28 frames per sample, "
                         "200 004 frames at the default)")
    ap.add_argument("--ml-steps", type=int, default=3000,
                    help="surrogate workload: mini-batch Adam steps")
    ap.add_argument("--skin", type=float, default=None,
                    help="Verlet skin (A); default 0.4 for one crystal (fastest measured), "
                         "1.3 for the sweep (hot replicas: measured 0.5-1.6, best 1.3-1.45), "
                         "1.0 for the surrogate")
    ap.add_argument("--profile-steps", type=int, default=256)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of known size (HBM counter scale)")
    ap.add_argument("--rocprof-summary", nargs="+", metavar="DIR",
                    help="print a markdown summary of rocprofv3 CSV output folders and exit")
    a = ap.parse_args()
    if a.rocprof_summary:
        print(rocprof_summary(a.rocprof_summary))
        return
    if a.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU: --gpus must be 1",
                          "n_gpus": a.gpus}))
        sys.exit(2)

    import torch
    from paper_1905_02521_amd import qtb, workloads as W

    torch.cuda.set_device(0)
    if a.skin is None:
        a.skin = (1.3 if a.workload.startswith("batched") else
                  1.0 if a.workload.startswith("surrogate") else 0.4)
    if a.workload == "qtb-vs-pimd":
        return pimd_compare_bench(a)
    if a.workload == "vdos":
        return vdos_bench(a)
    if a.workload == "npt":
        return npt_bench(a)
    if a.workload == "fir-modes":
        return fir_modes_bench(a)
    if a.workload.startswith("surrogate"):
        surrogate_bench(a)
        return
    batched = a.workload.startswith("batched")
    works = W.batched_sweep(int(a.workload.split("-")[1])) if batched else [W.workload(a.workload)]
    name = a.workload
    if a.cells:
        # the same workload on an n x n x n crystal
        w0 = works[0]
        if batched or w0.kind != "crystal":
            raise SystemExit("--cells applies to a single crystal workload")
        old_n = f"{w0.n_cells}x{w0.n_cells}x{w0.n_cells}"
        name = w0.name.replace(old_n, f"{a.cells}x{a.cells}x{a.cells}")
        works = [dataclasses.replace(w0, n_cells=a.cells, name=name)]
    pot = W.mgo_potential(skin=a.skin)
    fir = {"fp32": qtb.FIR_FP32, "bf16x3": qtb.FIR_BF16X3, "bf16": qtb.FIR_BF16,
           "fp64": qtb.FIR_FP64}[a.fir]
    prec = qtb.PREC_FP64 if fir == qtb.FIR_FP64 else qtb.PREC_FP32
    inputs, reps = [], []
    for w in works:
        beads, sp, box = W.crystal_inputs(w)
        inputs.append((beads, sp, box))
        reps.append(qtb.Replica(pos=beads, species=sp, T=w.T, gamma=w.gamma, dt=w.dt,
                                noise=w.noise, box=tuple(box), seed=w.seed, stream=w.stream))
    ctx = qtb.Context(qtb.pair_potential_dict(pot), reps, W.METAL_UNITS, prec=prec, fir=fir,
                      fir_block_K=a.K, obs_every=0, max_two_nf=max(max(w.two_nf, 2) for w in works),
                      noise_blocks=a.noise_blocks)
    for k, w in enumerate(works):
        if w.noise:
            ctx.build_filter(k, w.noise, w.two_nf)
    if a.decomposition:
        wpa, _, half = a.decomposition.partition(",")
        ctx.set_decomposition(int(wpa), half.strip() == "half")
    skins = None
    if batched and a.skin_full_T > 0:
        # per-replica list skin: the potential's at and above skin_full_T,
        # thinner for colder replicas (their atoms move less between rebuilds)
        skins = [max(min(a.skin, a.skin_min), min(a.skin, a.skin * math.sqrt(x.T / a.skin_full_T)))
                 for x in works]
        for k, sk in enumerate(skins):
            ctx.set_replica_skin(k, sk)
    w = works[0]
    beads, sp, box = inputs[0]
    ab_per_step = sum(b.shape[0] * b.shape[2] for b, _, _ in inputs)

    if a.copy_calibration:
        src = torch.empty(256 * 2**20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()

    # The coloured noise is made K steps at a time (white-noise rows and the FIR
    # contraction open every block).  The timed steps start on a block
    # boundary, so the timed region makes the noise of every step it runs:
    # after the warmup, untimed steps up to the next multiple of K.  With
    # --steps not a multiple of K the last block's noise is made for steps
    # beyond the timed ones too (a conservative figure).
    # The timed pattern (a.steps from a block boundary) is also run once
    # untimed, so that the graphs it replays are captured before the clock
    # starts, then the context steps on to the next block boundary.
    align = (-a.warmup) % a.K
    ctx.step(a.warmup + align)
    ctx.step(a.steps)
    ctx.step((-a.steps) % a.K)
    untimed = a.warmup + align + a.steps + (-a.steps) % a.K
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(a.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / a.steps
    value = ab_per_step * a.steps / (t1 - t0)
    wpa, half = ctx.decomposition()

    # per-kernel durations from HIP events on the library's stream
    ctx.profile(True)
    ctx.step(a.profile_steps)
    prof = ctx.profile_read()
    ctx.profile(False)
    f_ms, f_n = prof["forces"]
    force_ms = f_ms / max(f_n, 1)
    pairs = sum(unique_pairs(b, bx, pot.r_cut) for b, _, bx in inputs)
    flops = pairs * FLOPS_PER_PAIR
    achieved = flops / (force_ms * 1e-3) / 1e12
    fir_ms, fir_n = prof["fir"]
    D = 3 * ab_per_step
    fir_bytes = a.K * D * FIR_BYTES_PER_DOF_STEP
    fir_gbs = fir_bytes / (fir_ms / max(fir_n, 1) * 1e-3) / 1e9 if fir_n and not a.noise_blocks else None
    # HBM traffic from the committed counter record, valid only for this
    # workload and only while the pair kernel's source is unchanged
    traffic = stored_traffic() if name == "mgo-8x8x8-qtbpimd-P8-50K" else None
    phases = {k: {"ms_per_launch": v[0] / max(v[1], 1), "launches": v[1],
                  "ms_per_step": v[0] / a.profile_steps} for k, v in prof.items()}

    out = {
        "metric": "atom-bead-steps/s per GPU (forces+QTB noise+update)",
        "value": value,
        "unit": "atom-bead-steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == qtb.PREC_FP32 else "f64",
        "data": "synthetic (seeded rock-salt crystal, numpy PCG64 displacements)",
        "config": {"workload": name,
                   "replicas": len(works),
                   "atoms": sum(b.shape[2] for b, _, _ in inputs),
                   "atom_beads_per_step": ab_per_step,
                   "beads": sorted(set(x.P for x in works)),
                   "T_K": sorted(set(round(x.T, 2) for x in works)),
                   "noise": "QTB-PIMD kappa_P" if w.noise == 2 and not batched else
                            ("QTB theta" if not batched else "QTB theta (P=1) / kappa_P (P>1)"),
                   "two_nf": sorted(set(x.two_nf for x in works)), "fir": a.fir,
                   "noise_generator": "eq. 9 blocks" if a.noise_blocks else "streaming FIR",
                   "fir_block_K": a.K,
                   "untimed_steps": untimed,
                   "noise_blocks_in_timed_region": -(-a.steps // a.K),
                   "forces": "fp32" if prec == qtb.PREC_FP32 else "fp64", "state": "fp64",
                   "r_cut_A": pot.r_cut, "skin_A": pot.skin, "parallelism": "1 GPU",
                   "replica_skins_A": None if skins is None else
                   {"rule": f"min(skin, skin sqrt(T / {a.skin_full_T:g} K)), at least "
                            f"{min(a.skin, a.skin_min):g} A",
                    "min": round(min(skins), 3), "max": round(max(skins), 3)},
                   "force_decomposition": {"waves_per_atom": wpa, "half_bead_groups": half,
                                           "chosen_by": "pinned" if a.decomposition
                                           else "autotuner"}},
        "roofline": {"kernel": "pair forces", "bound": "alu", "achieved": achieved,
                     "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS,
                     "traffic": traffic["bytes"] if traffic else None,
                     "flops_per_launch": flops, "unique_pairs": pairs,
                     "flops_per_pair": FLOPS_PER_PAIR, "ms_per_launch": force_ms,
                     "slot_roofline": {
                         "slots_per_pair": SLOTS_PER_PAIR,
                         "achieved_slots_per_s": pairs * SLOTS_PER_PAIR / (force_ms * 1e-3),
                         "peak_slots_per_s": PEAK_LANE_SLOTS,
                         "frac": pairs * SLOTS_PER_PAIR / (force_ms * 1e-3) / PEAK_LANE_SLOTS}},
        "fir": None if a.noise_blocks else {
            "achieved_GBs": fir_gbs, "peak_GBs": PEAK_HBM_GBS,
            "frac": (fir_gbs / PEAK_HBM_GBS) if fir_gbs else None,
            "bytes_per_launch": fir_bytes, "ms_per_launch": fir_ms / max(fir_n, 1)},
        "phases": phases,
    }
    if batched and a.hc_blocks > 0:
        ctx.close()
        ctx = None
        out["heat_capacity"] = sweep_heat_capacity(works, inputs, pot, a)
    if not a.no_cpu:
        if batched:
            # smallest replica of each friction group, sharing the time budget
            picks = []
            for g in sorted(set(x.gamma for x in works)):
                ks = [k for k, x in enumerate(works) if x.gamma == g]
                picks.append(min(ks, key=lambda k: inputs[k][0].shape[2] * inputs[k][0].shape[0]))
            tot_ab, tot_t, parts = 0, 0.0, []
            for k in picks:
                cb = cpu_baseline(works[k], *inputs[k], pot, a.cpu_seconds / len(picks))
                parts.append(cb)
            # combined rate: total atom-bead-steps over total time
            n_ab = sum(p_["_ab"] for p_ in parts)
            t_all = sum(p_["_t"] for p_ in parts)
            out["cpu_baseline"] = {"value": n_ab / t_all, "unit": "atom-bead-steps/s",
                                   "cores": parts[0]["cores"], "kind": "oracle", **host_cpu(),
                                   "sample": "; ".join(p_["sample"] for p_ in parts)}
        else:
            cb = cpu_baseline(w, beads, sp, box, pot, a.cpu_seconds)
            cb.pop("_ab"); cb.pop("_t")
            out["cpu_baseline"] = cb
    if ctx is not None:
        ctx.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
