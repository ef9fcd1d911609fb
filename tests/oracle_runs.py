"""Cached oracle computations shared by the GPU parity tests (test helpers only)."""
from __future__ import annotations

import functools

import numpy as np

from oracle import dd, fem, geneo, pcg
from workloads import generate as gen

CASES = {
    "lam_2x2": lambda: gen.small_case("laminate", seed=21, nxy=(8, 6), n_ply=2, nparts=(2, 2, 1), nev=6),
    "lam_3x2x2_uneven": lambda: gen.small_case("laminate", seed=22, nxy=(12, 8), n_ply=3,
                                               nparts=(3, 2, 2), nev=8, uneven=True),
    "lam_ramp_traction": lambda: gen.small_case(
        "laminate", seed=23, nxy=(10, 4), n_ply=2, nparts=(2, 1, 1), nev=6, body=None,
        ramp=(3.0, 7.0, 0.17), traction=np.random.default_rng(5).normal(0, 0.01, 2 * 40 * 3), nrhs=2),
    "diff_2x2x2": lambda: gen.small_case("diffusion", seed=24, ne=(12, 10, 8), nparts=(2, 2, 2),
                                         overlap=2, threshold=0.15, nev_max=16),
    "diff_3x3x1": lambda: gen.small_case("diffusion", seed=25, ne=(15, 12, 6), nparts=(3, 3, 1),
                                         overlap=1, threshold=0.15, nev_max=12),
}


@functools.lru_cache(maxsize=None)
def workload(name):
    return CASES[name]()


@functools.lru_cache(maxsize=None)
def system(name):
    w = workload(name)
    Ke = fem.element_matrices(w)
    A, b, free = fem.assemble(w, Ke)
    return A, b, free, Ke


@functools.lru_cache(maxsize=None)
def geneo_run(name, coarse=True):
    w = workload(name)
    A, b, free, Ke = system(name)
    return geneo.GenEO(w, A, Ke, coarse=coarse, keep_all=True)


@functools.lru_cache(maxsize=None)
def geneo_run_shift(name, shift):
    w = workload(name)
    A, b, free, Ke = system(name)
    return geneo.GenEO(w, A, Ke, shift=shift, keep_all=True)


@functools.lru_cache(maxsize=None)
def pcg_run(name, rtol=1e-12):
    A, b, free, Ke = system(name)
    g = geneo_run(name)
    return pcg.pcg(A, b[:, 0], g.apply, rtol=rtol, maxit=2000)
