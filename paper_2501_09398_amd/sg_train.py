"""Training driver of the learned k-step surrogate (orchestration only).

Every numeric step runs in libkbatch: the trajectories are produced by the
plain GPU solver (the many-grid stencil advances all of a chunk's
trajectories with one kernel per step), and each optimisation step is one
kb_sg_train_step call (MFMA forward, loss, data and weight gradients,
Adam).  This module only chooses seeds, crops and learning rates.

Data (per trajectory i of a chunk): seed = base + i; T0 ~ U[323,343) and
P = U[0,1) plus 1-4 Gaussian hot spots, both drawn on the device by
kb_create of the surrogate problem with that seed; the state is recorded
after every k steps for `blocks` blocks, giving `blocks` training pairs
(T_jk, T_(j+1)k) that share P.  The initial weights are the seeded recipe
synth.surrogate_init.
Crops: C x C windows at uniform positions, a quarter of them pushed against
a randomly chosen grid edge so the replicate-padding border is learned.
"""
from __future__ import annotations

import os
import time
from dataclasses import dataclass

import numpy as np
import torch

import synth

from . import (F_P, F_RESID, F_SGSTATS, F_T, F_W, HEAT2D, HEAT2D_MULTI, HEAT2D_SURROGATE, HEAT_COEFFS, Problem)


# Weights of the network shipped with the package: written by this module's
# command line (python -m paper_2501_09398_amd.sg_train) with the defaults
# of TrainConfig; float32 little-endian, canonical order (19,393 values).
WEIGHTS_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "surrogate_k16.f32")


@dataclass
class TrainConfig:
    size: int = 512            # trajectory grid side
    trajectories: int = 2000
    chunk: int = 125           # trajectories generated at once
    blocks: int = 8            # k-step blocks recorded per trajectory
    k: int = 16
    s: float = 0.8
    crop: int = 128
    batch: int = 16
    steps: int = 8000
    lr: float = 5e-3
    lr_min: float = 5e-5
    edge_frac: float = 0.25
    seed: int = 1000
    init_seed: int = 7


def generate_chunk(cfg: TrainConfig, first: int, count: int, device=0):
    """(T0, P, Tk) device tensors [count*blocks][size][size] of one chunk."""
    n = cfg.size
    shape = [count] + [n, n] * count
    Ps, T0s = [], []
    for i in range(count):                  # the workload's seeded initial state, drawn by the library
        with Problem(HEAT2D_SURROGATE, (n, n), HEAT_COEFFS, cfg.seed + first + i, device=device) as q:
            T0s.append(q.read(F_T))
            Ps.append(q.read(F_P))
    states = []
    with Problem(HEAT2D_MULTI, shape, HEAT_COEFFS, 0, device=device) as p:
        p.write(F_T, np.concatenate([t.reshape(-1) for t in T0s]))
        p.write(F_P, np.concatenate([q.reshape(-1) for q in Ps]))
        buf = torch.empty(count * n * n, dtype=torch.float32, device=f"cuda:{device}")
        p.read_device(F_T, buf)
        states.append(buf.view(count, n, n).clone())
        for _ in range(cfg.blocks):
            p.run(cfg.k, 0)
            p.read_device(F_T, buf)
            states.append(buf.view(count, n, n).clone())
    P = torch.from_numpy(np.stack(Ps)).to(f"cuda:{device}")
    T0 = torch.cat([states[j] for j in range(cfg.blocks)], 0).contiguous()
    Tk = torch.cat([states[j + 1] for j in range(cfg.blocks)], 0).contiguous()
    Pf = P.repeat(cfg.blocks, 1, 1).contiguous()
    return T0, Pf, Tk


def sample_crops(rng, nfield, size, crop, batch, edge_frac):
    c = np.empty((batch, 3), np.int32)
    c[:, 0] = rng.integers(0, nfield, batch)
    c[:, 1] = rng.integers(0, size - crop + 1, batch)
    c[:, 2] = rng.integers(0, size - crop + 1, batch)
    for i in range(batch):
        if rng.random() < edge_frac:
            side = rng.integers(0, 4)
            if side == 0:
                c[i, 1] = 0
            elif side == 1:
                c[i, 1] = size - crop
            elif side == 2:
                c[i, 2] = 0
            else:
                c[i, 2] = size - crop
    return c


def train(cfg: TrainConfig, device=0, log=None):
    """Train from synth.surrogate_init(cfg.init_seed); returns (weights,
    history) with history a list of (step, loss, seconds)."""
    rng = np.random.default_rng(cfg.seed)
    coeffs = tuple(HEAT_COEFFS) + (cfg.s, 1e-3, cfg.k)
    hist = []
    t0 = time.perf_counter()
    nchunks = max(1, (cfg.trajectories + cfg.chunk - 1) // cfg.chunk)
    steps_per_chunk = max(1, cfg.steps // nchunks)
    with Problem(HEAT2D_SURROGATE, (64, 64, cfg.batch * cfg.crop * cfg.crop), coeffs, 0, device=device) as p:
        p.write(F_W, synth.surrogate_init(cfg.init_seed))
        step = 0
        for ch in range(nchunks):
            first = ch * cfg.chunk
            count = min(cfg.chunk, cfg.trajectories - first)
            T0, P, Tk = generate_chunk(cfg, first, count, device)
            for _ in range(steps_per_chunk):
                frac = step / max(1, cfg.steps - 1)
                lr = cfg.lr_min + 0.5 * (cfg.lr - cfg.lr_min) * (1 + np.cos(np.pi * min(1.0, frac)))
                crops = sample_crops(rng, T0.shape[0], cfg.size, cfg.crop, cfg.batch, cfg.edge_frac)
                loss = p.sg_train_step(T0, P, Tk, crops, cfg.crop, lr)
                if step % 100 == 0 or step == cfg.steps - 1:
                    hist.append((step, loss, time.perf_counter() - t0))
                    if log:
                        log(f"step {step} loss {loss:.4e} lr {lr:.2e} t {time.perf_counter() - t0:.1f}s")
                step += 1
            del T0, P, Tk
        w = p.read(F_W)
    return w, hist


def load_weights(path=WEIGHTS_FILE):
    w = np.fromfile(path, dtype="<f4")
    if w.size != 19393:
        raise ValueError(f"{path}: {w.size} values, expected 19393")
    return w


def plain_gpu(T0, P, steps, c=None, device=0):
    """`steps` plain float32 steps on the GPU (optionally with c replaced)."""
    coeffs = tuple(HEAT_COEFFS) if c is None else (c,) + tuple(HEAT_COEFFS[1:])
    with Problem(HEAT2D, T0.shape, coeffs, 0, device=device) as p:
        p.write(F_T, T0)
        p.write(F_P, P)
        p.run(steps, 0)
        return p.read(F_T)


def evaluate(weights, seeds, size=512, k=16, s=0.8, device=0, threshold=1e-3):
    """One surrogate block from held-out seeds against k plain float32 GPU
    steps, next to persistence (T_k = T0) and one explicit step of k*c
    ("big Euler").  Relative max-norms on T and on the increment T_k - T0.
    (The float32 plain stencil is within 1e-5 of float64 here; the tests
    compare against the float64 oracle.)"""
    rows = []
    coeffs = tuple(HEAT_COEFFS) + (s, threshold, k)
    c = HEAT_COEFFS[0]
    for sd in seeds:
        with Problem(HEAT2D_SURROGATE, (size, size), coeffs, sd, device=device) as p:
            T0, P = p.read(F_T), p.read(F_P)       # the seed's workload inputs, drawn on the device
            p.write(F_W, weights)
            p.run(k, 0)
            Tk = p.read(F_T).astype(np.float64)
            stats = p.read(F_SGSTATS)
            resid = float(p.read(F_RESID)[0])
        ref = plain_gpu(T0, P, k, device=device).astype(np.float64)
        inc = ref - T0
        euler = plain_gpu(T0, P, 1, c=k * c, device=device).astype(np.float64)

        def err(a):
            return (float(np.max(np.abs(a - ref)) / np.max(np.abs(ref))),
                    float(np.max(np.abs((a - T0) - inc)) / np.max(np.abs(inc))))
        e_sg, e_pers, e_eul = err(Tk), err(T0.astype(np.float64)), err(euler)
        rows.append({"seed": sd, "surrogate_T": e_sg[0], "surrogate_inc": e_sg[1],
                     "persistence_T": e_pers[0], "persistence_inc": e_pers[1],
                     "euler_T": e_eul[0], "euler_inc": e_eul[1], "residual": resid,
                     "fallback": int(stats[1])})
    return rows


if __name__ == "__main__":
    import argparse
    import json
    ap = argparse.ArgumentParser(description="train the k-step surrogate on GPU-generated trajectories")
    ap.add_argument("--trajectories", type=int, default=TrainConfig.trajectories)
    ap.add_argument("--steps", type=int, default=TrainConfig.steps)
    ap.add_argument("--lr", type=float, default=TrainConfig.lr)
    ap.add_argument("--out", default=WEIGHTS_FILE)
    a = ap.parse_args()
    cfg = TrainConfig(trajectories=a.trajectories, steps=a.steps, lr=a.lr)
    w, hist = train(cfg, log=lambda m: print(m, flush=True))
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    w.astype("<f4").tofile(a.out)
    print(json.dumps({"config": cfg.__dict__, "history": hist[-3:], "eval": evaluate(w, [900001, 900002])}))
