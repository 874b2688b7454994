"""Training data and training loop of the learned force surrogate (the
library's qtb_ml_* calls): frames from the method's own QTB and QTB-PIMD runs
of the pair potential, labelled by that potential, and mini-batch Adam on the
GPU.  Argument marshalling and bookkeeping only: the runs, labels,
descriptors, network, loss, gradient and Adam step are the library's
kernels."""
from __future__ import annotations

import math

import numpy as np

from . import qtb, workloads as W


def qtb_frames(pot, conditions, n_frames, every=40, warm=2000, n_cells=4, gamma=1e-3,
               two_nf=512, seed=0):
    """Frames of the n_cells^3 rock-salt crystal from one batched context that
    runs one replica per (T, P) in `conditions`: QTB (theta noise, eq. 1) for
    P = 1, QTB-PIMD (kappa_P noise, eq. 10-12) for P > 1, production
    precision.  After `warm` steps, every `every` steps each bead of each
    replica is one frame (n_frames samples per replica).  Labels are the pair
    potential's forces and energy of that bead configuration.

    Returns (positions [M][3][N], forces [M][3][N], energies [M], species,
    box, tags [M] of (T, P))."""
    pos, sp, box = W.rocksalt(n_cells)
    reps = []
    for k, (T, P) in enumerate(conditions):
        base = W.displaced(pos, 0.0421, 1000 + seed * 100 + k)
        beads = (base[None] if P == 1 else
                 np.stack([W.displaced(base, 0.005, 2000 + seed * 1000 + 10 * k + b)
                           for b in range(P)]))
        reps.append(qtb.Replica(pos=beads, species=sp, T=float(T), gamma=gamma, dt=1.0,
                                noise=1 if P == 1 else 2, box=tuple(box), seed=500 + seed,
                                stream=k))
    # one fixed force decomposition: the same frames on every run
    ctx = qtb.Context(qtb.pair_potential_dict(pot), reps, dict(W.METAL_UNITS),
                      prec=qtb.PREC_FP32, fir=qtb.FIR_BF16X3, max_two_nf=two_nf,
                      autotune=False)
    for k, (_, P) in enumerate(conditions):
        ctx.build_filter(k, 1 if P == 1 else 2, two_nf)
    ctx.step(warm)
    frames, forces, energies, tags = [], [], [], []
    for _ in range(n_frames):
        ctx.step(every)
        for k, (T, P) in enumerate(conditions):
            r, _, _ = ctx.get_state(k)
            f, e = ctx.evaluate(k)
            for b in range(P):
                frames.append(r[b])
                forces.append(f[b])
                energies.append(e[b])
                tags.append((float(T), int(P)))
    ctx.close()
    return (np.array(frames), np.array(forces), np.array(energies), sp, np.asarray(box),
            tags)


def _ctx(pot, frames, sp, box, train, ml_r_cut):
    reps = [qtb.Replica(pos=f[None], species=sp, T=300.0, gamma=1e-3, dt=1.0, noise=0,
                        box=tuple(box), seed=1, stream=k) for k, f in enumerate(frames)]
    return qtb.Context(qtb.pair_potential_dict(pot), reps, dict(W.METAL_UNITS),
                       prec=qtb.PREC_FP32, fir=qtb.FIR_FP32, ml_r_cut=ml_r_cut,
                       ml_train=train)


def train(model, pot, frames, forces, energies, sp, box, steps, batch=256, lr=(3e-3, 1e-3),
          w_E=1.0, w_F=1.0, ml_r_cut=6.0, seed=0, max_contexts=64):
    """Mini-batch Adam: the training frames are shuffled once and dealt into
    n_b = ceil(n / batch) batches of equal size floor(n / n_b) (batch q holds
    the shuffled frames q, q + n_b, ...; at most n_b - 1 frames are left
    out); step k uses batch k mod n_b with learning rate lr[0] for the first
    two thirds of the steps and lr[1] after.  Up to max_contexts batches each
    keep a context of their own; beyond that one context takes the batches in
    turn (the frames and labels stay on the GPU and each batch is loaded into
    the context's state arrays, its lists and forces following: about 8 ms
    per load of 256 frames of 512 atoms).  The input normalisation and energy
    offsets are fitted on the first batch.  Returns the loss of every step."""
    import torch
    order = np.random.default_rng(seed).permutation(len(frames))
    n_b = max(1, math.ceil(len(frames) / batch))
    size = len(frames) // n_b
    idx = [torch.as_tensor(order[q::n_b][:size], device="cuda") for q in range(n_b)]
    d_for = torch.as_tensor(forces, dtype=torch.float64, device="cuda")
    d_en = torch.as_tensor(energies, dtype=torch.float64, device="cuda")

    def labels_of(q, c):
        lab = (d_en.index_select(0, idx[q]).contiguous(),
               d_for.index_select(0, idx[q]).reshape(-1).contiguous())
        c.torch_stream.wait_stream(torch.cuda.current_stream())
        return lab

    stream = n_b > max_contexts
    ctxs, labels = [], []
    losses = []
    try:
        if stream:
            d_pos = torch.as_tensor(frames, dtype=torch.float64, device="cuda")
            ctxs.append(_ctx(pot, frames[order[0::n_b][:size]], sp, box, True, ml_r_cut))
            labels.append(labels_of(0, ctxs[0]))
        else:
            for q in range(n_b):
                ctxs.append(_ctx(pot, frames[order[q::n_b][:size]], sp, box, True, ml_r_cut))
                labels.append(labels_of(q, ctxs[q]))
        ctxs[0].ml_fit_norm(model, labels[0][0])
        loaded = 0
        for k in range(steps):
            q = k % n_b
            if stream:
                c = ctxs[0]
                if loaded != q:
                    c.set_positions(d_pos.index_select(0, idx[q]))
                    labels[0] = labels_of(q, c)
                    loaded = q
                lab = labels[0]
            else:
                c, lab = ctxs[q], labels[q]
            rate = lr[0] if k < (2 * steps) // 3 else lr[1]
            losses.append(c.ml_train_step(model, lab[0], lab[1], w_E, w_F, rate))
    finally:
        for c in ctxs:
            c.close()
    return np.array(losses)


def errors(model, pot, frames, forces, energies, sp, box, ml_r_cut=6.0, chunk=256):
    """Force and energy errors of the surrogate against the labels: RMS of
    the force components (eV/A), the same relative to the labels' RMS, and
    the RMS energy error per atom (eV).  The frames go through one context
    of chunk replicas (and one for the last, shorter chunk)."""
    import torch
    err = ref = 0.0
    de = []
    N = len(sp)
    n_full = (len(frames) // chunk) * chunk
    spans = [(q0, chunk) for q0 in range(0, n_full, chunk)]
    if n_full < len(frames):
        spans.append((n_full, len(frames) - n_full))
    ctxs = {}
    try:
        for q0, m in spans:
            sub = frames[q0:q0 + m]
            if m not in ctxs:
                ctxs[m] = _ctx(pot, sub, sp, box, False, ml_r_cut)
            else:
                ctxs[m].set_positions(torch.as_tensor(sub, dtype=torch.float64, device="cuda"))
            c = ctxs[m]
            for k in range(m):
                f, e, _, _ = c.ml_evaluate(model, k)
                err += float(np.sum((f[0] - forces[q0 + k]) ** 2))
                ref += float(np.sum(forces[q0 + k] ** 2))
                de.append((e[0] - energies[q0 + k]) / N)
    finally:
        for c in ctxs.values():
            c.close()
    n = forces.size
    return math.sqrt(err / n), math.sqrt(err / ref), float(np.sqrt(np.mean(np.square(de))))
