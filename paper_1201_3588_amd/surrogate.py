"""Learned PAH emission step: dataset from the exact solver, training, and the
surrogate-in-the-loop solve with exact fallback on out-of-distribution cells.

Orchestration only: the exact solver, the dataset transforms and
normalisation, every forward/backward product, the loss, Adam and inference
run in libmcrt.so kernels; torch supplies buffers, the batch permutation and
row gathers.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from .pah import PahMLP, PahSolver, exact_fallback

N_BANDS = 17


def band_error(pred, exact, n_bands=N_BANDS):
    """Per-cell flux-weighted band error sum_b |F^_b - F_b| / sum_b F_b."""
    pb, eb = pred[:, :n_bands], exact[:, :n_bands]
    return (pb - eb).abs().sum(1) / eb.sum(1)


def init_params(n_in, n_h, n_out, seed):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases."""
    g = np.random.default_rng(seed)
    p = {}
    for name, (o, i) in dict(W1=(n_h, n_in), W2=(n_h, n_h), W3=(n_out, n_h)).items():
        lim = 1.0 / math.sqrt(i)
        p[name] = g.uniform(-lim, lim, size=(o, i)).astype(np.float32)
    p["b1"] = np.zeros(n_h, np.float32)
    p["b2"] = np.zeros(n_h, np.float32)
    p["b3"] = np.zeros(n_out, np.float32)
    return p


class Surrogate:
    """Exact solver + network for one PAH species."""

    def __init__(self, solver: PahSolver, n_h=256, batch=2048, seed=4):
        self.solver = solver
        self.batch = batch
        self.net = PahMLP(solver.n_lambda + 1, n_h, solver.n_out, batch=batch, device=solver.device)
        self.net.load(init_params(solver.n_lambda + 1, n_h, solver.n_out, seed))
        self.seed = seed

    def exact(self, J, chunk=1 << 18):
        """Exact outputs [n, n_out] (float64) and absorbed powers for fields J [n, nl]."""
        n = int(J.shape[0])
        out = torch.empty((n, self.solver.n_out), dtype=torch.float64, device=J.device)
        pabs = torch.empty(n, dtype=torch.float64, device=J.device)
        for a in range(0, n, chunk):
            b = min(n, a + chunk)
            o, _, p = self.solver.solve(J[a:b])
            out[a:b] = o
            pabs[a:b] = p
        return out, pabs

    def fit(self, J, out, pabs, epochs=30, lr=2e-3, log=None):
        """Train on solved cells (J float32 [n, nl] device).  Cosine learning rate."""
        X, Y = self.net.prepare(self.solver, J, out, pabs)
        n = int(X.shape[0])
        B = self.batch
        steps_per_epoch = n // B
        total = epochs * steps_per_epoch
        g = torch.Generator(device=J.device)
        g.manual_seed(self.seed)
        step = 0
        hist = []                      # loss of the first batch, then at each epoch end
        for ep in range(epochs):
            perm = torch.randperm(n, generator=g, device=J.device)
            for k in range(steps_per_epoch):
                idx = perm[k * B:(k + 1) * B]
                step += 1
                lr_t = lr * 0.5 * (1.0 + math.cos(math.pi * (step - 1) / total))
                self.net.train_step(X.index_select(0, idx), Y.index_select(0, idx), lr_t, step)
                if step == 1:
                    hist.append(self.net.loss())
            hist.append(self.net.loss())
            if log:
                log(f"epoch {ep} loss {hist[-1]:.5f}")
        return hist

    def predict(self, J, in_margin=0.5, balance_tol=0.02):
        return self.net.infer(self.solver, J, in_margin, balance_tol)

    def solve(self, J, in_margin=0.5, balance_tol=0.02):
        """Surrogate in the loop: network everywhere, exact solver on flagged cells."""
        out, ood, pabs = self.predict(J, in_margin, balance_tol)
        idx = exact_fallback(self.solver, J, ood, out)
        return out, ood, pabs, idx
