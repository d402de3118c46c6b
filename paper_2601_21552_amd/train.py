"""Training of the learned branching scorer from the splitter's own traces.

The splitter records, at decision nodes of its static walk, the features of
the top candidate variables and a one-step lookahead label for each
(``Context.trace``).  The perceptron is regressed on those labels, centred
and scaled per node, since only the order of the candidates within a node
matters.  Forward, backward and Adam run in the library's kernels
(``api.Mlp``); this module only shuffles rows on the host and moves batches
to the device.
"""
from __future__ import annotations

import time

import numpy as np

from . import api


def bf16_bits(x: np.ndarray) -> np.ndarray:
    """float32 -> bfloat16 bit patterns, round to nearest, ties to even."""
    u = np.ascontiguousarray(x, np.float32).view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    nan = np.isnan(np.asarray(x, np.float32))
    r = np.where(nan, (u >> 16) | 0x40, r)
    return r.astype(np.uint16)


def node_targets(labels: np.ndarray, nodes: np.ndarray) -> np.ndarray:
    """Labels centred on their node's mean and divided by its standard
    deviation (plus 0.05, so that flat nodes stay near zero)."""
    labels = np.asarray(labels, np.float64)
    _, inv = np.unique(nodes, return_inverse=True)
    cnt = np.bincount(inv).astype(np.float64)
    mean = np.bincount(inv, labels) / cnt
    var = np.bincount(inv, (labels - mean[inv]) ** 2) / cnt
    return ((labels - mean[inv]) / (np.sqrt(var[inv]) + 0.05)).astype(np.float32)


def collect(ctx: "api.Context", cnfs, k: int, candidates: int = 16, every: int = 1,
            depth: int = 48, max_cubes: int = 20000):
    """Traces of several CNF batches, concatenated.  Node ids are made
    unique across batches (batch index in bits 56 and up)."""
    fs, ls, ns = [], [], []
    for b, cnf in enumerate(cnfs):
        f, lab, n = ctx.trace(cnf, k=k, candidates=candidates, every=every, depth=depth,
                              max_cubes=max_cubes)
        fs.append(f)
        ls.append(lab)
        ns.append(n | (np.uint64(b) << np.uint64(56)))
    return np.concatenate(fs), np.concatenate(ls), np.concatenate(ns)


def train(ctx: "api.Context", feats: np.ndarray, targets: np.ndarray, epochs: int = 8,
          batch: int = 1024, lr: float = 2e-3, seed: int = 0, init=None, log=None):
    """Adam on the mean squared error; returns (Mlp, per-epoch mean loss).
    init: flat initial parameters (default: He initialisation from seed)."""
    import torch
    rng = np.random.Generator(np.random.PCG64(seed))
    if init is None:
        init = _he_init(rng)
    mlp = api.Mlp(ctx, init)
    dev = mlp.dev
    n = len(targets)
    if n == 0:
        raise ValueError("no training rows")
    xb = bf16_bits(feats).view(np.int16)
    history = []
    for ep in range(epochs):
        perm = rng.permutation(n)
        x_dev = torch.from_numpy(np.ascontiguousarray(xb[perm])).to(dev).view(torch.bfloat16)
        t_dev = torch.from_numpy(np.ascontiguousarray(targets[perm], np.float32)).to(dev)
        losses = []
        t0 = time.perf_counter()
        for s in range(0, n - batch + 1 if n >= batch else 1, batch):
            e = min(n, s + batch)
            x = x_dev[s:e]
            t = t_dev[s:e]
            y, a1, a2 = mlp.forward(x)
            mlp.backward(x, a1, a2, y, t)
            mlp.adam(lr=lr)
            losses.append((y, t))
        torch.cuda.synchronize()
        ep_loss = float(np.mean([np.mean((y.cpu().numpy() - t.cpu().numpy()) ** 2) for y, t in losses]))
        history.append(ep_loss)
        if log:
            log(f"epoch {ep}: loss {ep_loss:.4f} ({time.perf_counter() - t0:.2f} s, {len(losses)} steps)")
    return mlp, history


def _he_init(rng: np.random.Generator, F: int = 16, H: int = 128) -> np.ndarray:
    p = {
        "W1": rng.standard_normal((F, H)) * np.sqrt(2.0 / F),
        "b1": np.zeros(H),
        "W2": rng.standard_normal((H, H)) * np.sqrt(2.0 / H),
        "b2": np.zeros(H),
        "w3": rng.standard_normal(H) * np.sqrt(1.0 / H),
        "b3": np.zeros(1),
    }
    return api.mlp_flatten(p)


def save(mlp: "api.Mlp", path: str):
    np.save(path, mlp.params())


def load(ctx: "api.Context", path: str) -> "api.Mlp":
    return api.Mlp(ctx, np.load(path, allow_pickle=False))
