"""Learned initial guess for the ensemble solve.

A POD basis of r modes is built from solutions the solver itself produced
(method of snapshots on the device), a 10 -> 256 -> 256 -> 32 GELU network is
trained on the device to map the KL inputs y to the standardised POD
coefficients, and its prediction, lifted back through the basis, seeds CG.
CG itself still decides convergence, so a poor prediction costs iterations,
never accuracy.  All arithmetic runs in the library's kernels; this class
only sequences the calls and owns the tensors.
"""
from __future__ import annotations

import numpy as np
import torch

from . import ens


class LearnedGuess:
    def __init__(self, r: int = 32, device="cuda"):
        if r != ens.MLP_OUT:
            raise ValueError(f"the network predicts {ens.MLP_OUT} coefficients; r must equal it")
        self.r = r
        self.device = device
        self.Phi = self.mu = self.sd = self.params = None
        self.lam = None
        self.loss = None

    def fit_basis(self, S: torch.Tensor, eig_seed: int, oversample: int = 32, eig_iters: int = 12,
                  common_scale: bool = True):
        """S [n][m] FP64 snapshots (device).  Returns the network targets
        [m][r] (FP32): the snapshots' POD coefficients centred and divided by
        one common scale (the largest coefficient deviation), so the training
        loss weighs each coefficient by its share of the guess's error, or
        with common_scale=False each by its own deviation."""
        m = S.shape[1]
        G = ens.pod_gram(S)
        k = min(m, self.r + oversample)
        start = torch.as_tensor(np.random.default_rng(eig_seed).standard_normal((m, k)), device=self.device)
        V, self.lam = ens.pod_eig(G, self.r, start, eig_iters)
        self.Phi = ens.pod_basis(S, V, self.lam)
        C = ens.pod_project(self.Phi, S)
        self.mu, self.sd, T = ens.pod_standardize(C, common=common_scale)
        return T

    def fit_network(self, xi: torch.Tensor, T: torch.Tensor, steps: int, init_seed: int, order_seed: int,
                    batch: int = 256, lr: float = 1e-3, halvings: int = 0):
        """xi [m][10] FP32, T [m][r] FP32 (device).  Adam on shuffled
        mini-batches (a fresh permutation per epoch); the steps are split into
        halvings + 1 equal stages with the learning rate halved per stage."""
        m = xi.shape[0]
        self.params = ens.mlp_init(init_seed, self.device)
        am = torch.zeros_like(self.params)
        av = torch.zeros_like(self.params)
        epochs = (steps * batch + m - 1) // m
        idx = np.concatenate([np.random.default_rng(order_seed + e).permutation(m) for e in range(epochs)])
        idx = torch.as_tensor(idx[:steps * batch].astype(np.int32), device=self.device)
        self.loss = torch.zeros(steps, dtype=torch.float32, device=self.device)
        stages = halvings + 1
        bounds = [steps * i // stages for i in range(stages + 1)]
        for i in range(stages):
            a, b = bounds[i], bounds[i + 1]
            if b > a:
                ens.mlp_train(self.params, am, av, a, xi, T, batch, idx[a * batch:b * batch], lr * 0.5 ** i,
                              loss=self.loss[a:b])
        return self.loss

    def guess(self, xi32: torch.Tensor, x0: torch.Tensor | None = None) -> torch.Tensor:
        """Initial guesses [n][s] FP64 for KL inputs xi32 [s][10] FP32."""
        c = ens.mlp_forward(self.params, xi32)
        return ens.pod_reconstruct(self.Phi, c, self.mu, self.sd, x0=x0)
