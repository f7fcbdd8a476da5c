"""Seeded synthetic workloads shared by the tests, the smoke check and the
benchmark.

This module holds no arithmetic of the method: it only names the problem
configurations and draws the random inputs.  Both the GPU library and the CPU
oracle receive the same arrays from here, so neither re-implements a random
number generator.

The random variables are the Karhunen-Loeve inputs y_i ~ U[-1, 1] of the
diffusion coefficient (Sec. 4 of Phipps et al.), drawn as
``numpy.random.default_rng(seed).uniform(-1, 1, (s, M))`` (row e = sample e).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    N: int             # elements per axis of the unit-cube hex mesh
    s: int             # ensemble size
    M: int             # KL terms
    sigma: float       # standard deviation in front of the KL sum
    rtol: float        # relative residual target |b - A x| <= rtol |b|
    mixed: bool        # FP32 inner CG inside FP64 iterative refinement
    seed: int
    L: float = 1.0     # correlation length
    kappa0: float = 1.0
    f: float = 1.0     # constant source term
    notes: str = ""

    @property
    def n(self) -> int:
        return (self.N + 1) ** 3

    @property
    def nnz(self) -> int:
        return (3 * self.N + 1) ** 3

    def xi(self, count: int | None = None, seed: int | None = None) -> np.ndarray:
        return draw_xi(self.seed if seed is None else seed, self.s if count is None else count, self.M)


def draw_xi(seed: int, count: int, M: int) -> np.ndarray:
    """KL inputs y ~ U[-1,1]^M, one row per sample."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=(count, M))


def draw_vector(seed: int, shape, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    return np.random.default_rng(seed).uniform(lo, hi, size=shape)


# The five workloads of the measurement plan.
SMALL = Workload("q1_16cube_s4_fp64", N=16, s=4, M=3, sigma=0.1, rtol=1e-10, mixed=False, seed=1000,
                 notes="16^3 elements, 4913 nodes, Jacobi-CG to 1e-10, FP64")
MID = Workload("q1_64cube_s16_fp64", N=64, s=16, M=10, sigma=0.2, rtol=1e-10, mixed=False, seed=1001,
               notes="64^3 elements, 274625 nodes, Jacobi-CG to 1e-10, FP64")
HEADLINE = Workload("q1_128cube_s32_mixed", N=128, s=32, M=10, sigma=0.3, rtol=1e-8, mixed=True, seed=1002,
                    notes="128^3 elements, 2146689 nodes, FP32 CG inside FP64 refinement to 1e-8")
LEARNED = Workload("q1_64cube_s32_learned", N=64, s=32, M=10, sigma=0.2, rtol=1e-8, mixed=False, seed=1005,
                   notes="POD r=32 from 2048 solves; MLP 10-256-256-32 initial guess")

# The nonlinear problem of Sec. 4 with the advection and reaction terms on:
# the headline samples (128^3, s = 32, M = 10, sigma = 0.3, seed 1002),
# alpha v.grad u with v = (1,1,1)/sqrt(3) and beta u^2, Newton to 1e-8.
NEWTON = Workload("q1_128cube_s32_newton", N=128, s=32, M=10, sigma=0.3, rtol=1e-8, mixed=False, seed=1002,
                  notes="128^3, s=32, alpha=10, beta=100: Newton with multigrid-preconditioned GMRES(30)")
NEWTON_ALPHA = 10.0
NEWTON_BETA = 100.0
NEWTON_VEL = (3 ** -0.5, 3 ** -0.5, 3 ** -0.5)
NEWTON_LIN_RTOL = 3e-3   # fixed forcing: measured fastest of 1e-2, 3e-3, 1e-3, 1e-4 at 128^3, s = 32
NEWTON_ETA_MAX = 0.3     # Eisenstat-Walker forcing: eta_0 = eta_max
NEWTON_RESTART = 30

BATCH_MESHES = (32, 48, 64, 96)
BATCH_GROUPS = 256
BATCH_MESH_SEED = 1003
BATCH_XI_SEED = 1004
BATCH_TUNE_SEED = 1010   # autotuner trial samples, one draw per mesh size
BATCH_SIGMA = 0.2
BATCH_M = 10
BATCH_RTOL = 1e-8

LEARNED_TRAIN_SEED = 1005
LEARNED_TEST_SEED = 1006
LEARNED_INIT_SEED = 1007
LEARNED_TRAIN = 2048
LEARNED_TEST = 1024


def batch_meshes(groups: int = BATCH_GROUPS, seed: int = BATCH_MESH_SEED) -> np.ndarray:
    """Mesh size N of each sample group, uniform over the four batch meshes."""
    rng = np.random.default_rng(seed)
    return np.asarray(BATCH_MESHES)[rng.integers(0, len(BATCH_MESHES), size=groups)]
