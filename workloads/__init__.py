"""Seeded synthetic workloads: configuration presets and random draws.

This module is shared by the HIP library's tests and benchmark and by the CPU
oracle.  It holds workload descriptions and seeded standard-normal draws only,
and none of the method's arithmetic: the random numbers the method consumes
(truth perturbation, background and observation perturbations, Gaussian sketch
matrices) are drawn here and handed to both implementations as inputs, so that
both index the same numbers.

Layout of the per-problem normal vector (length 1 + (L+1)(n+p)), with p the
number of observations and L the number of perturbed members:

    [0]                         truth spin-up perturbation z (one value)
    [1 + j*n : 1 + (j+1)*n]     xi_j,  j = 0..L   background draws (xi_0: control)
    [1 + (L+1)*n + j*p : ...]   eta_j, j = 0..L   observation draws (eta_0: truth obs error)

The problems are identical-twin Lorenz-96 experiments (numerical-experiments
section of the paper); the paper uses synthetic data only, and so do these.
"""
from __future__ import annotations

import copy

import numpy as np

# Model / assimilation parameters.  Keys:
#   n, nsteps (window N), F, dt, spinup (truth spin-up steps), spin_pert_std,
#   obs_dt (observation every obs_dt steps, time 0 excluded), obs_dx, obs_x0
#   (observed variables i = obs_x0 + q*obs_dx), sigma_o (R = sigma_o^2 I),
#   sigma_b, len_b, b_kind, diff_steps (B = sigma_b^2 C: b_kind "gauss", the
#   cyclic Gaussian correlation of length len_b; or "diffusion", the
#   diffusion-based correlation with Daley length-scale len_b and diff_steps
#   diffusion steps),
#   members (L perturbed members; member 0 is the control),
#   ell, k (sketch columns / retained rank), q (Nystrom passes), theta ('mid'),
#   rtol, maxit (PCG).
_BASE = dict(F=8.0, dt=0.025, spinup=1000, spin_pert_std=0.1, obs_x0=0,
             sigma_o=0.5, sigma_b=1.0, b_kind="gauss", diff_steps=0, q=1, theta="mid", seed=0, problem_id=0)

CONFIGS = {
    # Plain FP64, n = 40; every 2nd variable every 5 steps; PCG exactly 50 iterations.
    "C1": dict(_BASE, n=40, nsteps=20, obs_dt=5, obs_dx=2, len_b=2.0, members=10,
               ell=10, k=10, rtol=0.0, maxit=50),
    # n = 1024, all variables observed every 5 steps, 64 members, k = 32.
    "C2": dict(_BASE, n=1024, nsteps=40, obs_dt=5, obs_dx=1, len_b=8.0, members=64,
               ell=32, k=32, rtol=1e-6, maxit=2000),
    # n = 4096, every 2nd variable every 4 steps, 128 members, k = 64.
    "C3": dict(_BASE, n=4096, nsteps=40, obs_dt=4, obs_dx=2, len_b=8.0, members=128,
               ell=64, k=64, rtol=1e-6, maxit=2000),
    # The paper's own set-up (numerical-experiments section): n = 1500, a
    # 10-step window, direct observations of 50 variables (every 30th) at 3
    # times (steps 3, 6, 9: p = 150), sigma_o = 0.05, sigma_b = 0.8, the
    # diffusion-based B with D = 6 and M = 10, L = ell = 20 members, k = 20
    # (k = 15 with oversampling in the sensitivity study).
    "paper": dict(_BASE, n=1500, nsteps=10, obs_dt=3, obs_dx=30, sigma_o=0.05, sigma_b=0.8,
                  b_kind="diffusion", len_b=6.0, diff_steps=10, members=20, ell=20, k=20,
                  rtol=1e-6, maxit=2000),
}


def config(name: str, **over) -> dict:
    """A copy of preset `name` with keyword overrides."""
    c = copy.deepcopy(CONFIGS[name])
    c.update(over)
    return c


def obs_counts(cfg: dict) -> tuple[int, int]:
    """(number of observation times, number of observed variables)."""
    nt = cfg["nsteps"] // cfg["obs_dt"]
    x0, dx, n = cfg["obs_x0"], cfg["obs_dx"], cfg["n"]
    nv = 0 if x0 >= n else (n - 1 - x0) // dx + 1
    return nt, nv


def n_normals(cfg: dict) -> int:
    nt, nv = obs_counts(cfg)
    return 1 + (cfg["members"] + 1) * (cfg["n"] + nt * nv)


def _rng(seed: int, problem_id: int, stream: int) -> np.random.Generator:
    # Counter-based generator keyed by (seed, problem, stream): independent
    # streams that any run reproduces exactly.
    key = (int(seed) & 0xFFFFFFFF) | ((int(problem_id) & 0xFFFFFF) << 32) | ((int(stream) & 0xFF) << 56)
    return np.random.Generator(np.random.Philox(key=key))


def problem_normals(cfg: dict) -> np.ndarray:
    """Standard normals for one EDA problem (layout in the module docstring)."""
    return _rng(cfg["seed"], cfg["problem_id"], 0).standard_normal(n_normals(cfg))


def ensemble_normals(cfg: dict, draw: int) -> np.ndarray:
    """Normals of one problem whose control part (truth perturbation, xi_0,
    eta_0) is that of problem_normals(cfg) and whose member perturbations
    (xi_j, eta_j, j >= 1) are draw `draw` of a separate stream (9): the same
    control problem with another ensemble, as in repeated experiments with
    different ensemble instances."""
    z = problem_normals(cfg)
    nt, nv = obs_counts(cfg)
    n, L, p = cfg["n"], cfg["members"], nt * nv
    fresh = _rng(cfg["seed"], cfg["problem_id"] * 4096 + draw, 9).standard_normal(L * (n + p))
    z[1 + n:1 + (L + 1) * n] = fresh[:L * n]
    z[1 + (L + 1) * n + p:] = fresh[L * n:]
    return z


def gaussian_matrix(cfg: dict, rows: int, cols: int, stream: int = 5, draw: int | None = None) -> np.ndarray:
    """A seeded standard-Gaussian matrix stored column-major as an array of
    shape (cols, rows): row c of the array is column c of the matrix.  With
    `draw`, draw number `draw` of a family of independent such matrices (keyed
    as ensemble_normals keys its draws)."""
    pid = cfg["problem_id"] if draw is None else cfg["problem_id"] * 4096 + draw
    return _rng(cfg["seed"], pid, stream).standard_normal((cols, rows))


def uneven_problems(count: int = 256, seed: int = 0) -> list[dict]:
    """Independent EDA problems of uneven shape: n from {40,128,512,1024,2048},
    window from {10,20,40}, members from 8..64, k = min(32, members); other
    parameters as the n = 1024 preset (length scale 2 for n = 40)."""
    rng = _rng(seed, 0, 8)
    out = []
    for pid in range(count):
        n = int(rng.choice([40, 128, 512, 1024, 2048]))
        N = int(rng.choice([10, 20, 40]))
        L = int(rng.integers(8, 65))
        k = min(32, L)
        c = config("C2", n=n, nsteps=N, members=L, ell=k, k=k, problem_id=pid + 1,
                   len_b=2.0 if n == 40 else 8.0, seed=seed)
        out.append(c)
    return out


def mlp_init_normals(count: int, seed: int = 0) -> np.ndarray:
    """Standard normals for the learned-sketch network's initialisation
    (stream 6), one per parameter."""
    return _rng(seed, 0, 6).standard_normal(count).astype(np.float32)


def data_order(count: int, epoch: int, seed: int = 0) -> np.ndarray:
    """A permutation of the training samples for one epoch (stream 7)."""
    return _rng(seed, epoch, 7).permutation(count)


LEARNED_SPLITS = {"train": (1, 20000), "val": (20001, 20500), "test": (30001, 30256)}


def learned_problem(problem_id: int, members: int = 64, seed: int = 0) -> dict:
    """A problem of the n = 1024 preset for the learned sketch (train, validation
    and test ids as in LEARNED_SPLITS)."""
    return config("C2", members=members, ell=min(32, members), k=min(32, members), problem_id=problem_id, seed=seed)
