"""Cached oracle computations shared by the GPU parity tests (test helpers only)."""
from __future__ import annotations

import dataclasses
import functools

import numpy as np

from oracle import dd, fem, geneo, pcg  # noqa: F401
from workloads import generate as gen

# Cases small enough for the oracle in seconds; their local bands are at most 3
# tiles wide, so they exercise the narrowest kernel instantiations.
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

# Cases whose subdomain boxes give the band widths of the full-size
# configurations (slow: dense oracle factors of 5k-11k rows):
#  diff_wide10  local band 10 tiles (the FP64 sweep with 20 slots per thread,
#               as the SPE10-shaped diffusion), pencil band 10 tiles;
#  lam_wide12   local band 12 tiles (24 slots, as the ramped laminate), pencil
#               band 13 tiles (an 18-slot ring of the eigen block solves);
#  lam_wide17   local band 17 tiles (34 slots of the 512-thread sweep;
#               forced, the 16-column matrix-core kernel with one live column);
#               compared one-level and with the zero-energy-mode coarse space
#               (no dense eigensolve);
#  lam_wide22   local band 22 tiles, the widest of the 12-ply laminate: the
#               512-thread FP64 sweep at its 44-slot limit; one-level only.
WIDE = {
    "diff_wide10": lambda: gen.small_case("diffusion", seed=31, ne=(32, 16, 16), nparts=(2, 1, 1), overlap=2,
                                          threshold=0.15, nev_max=16),
    "lam_wide12": lambda: gen.small_case("laminate", seed=32, nxy=(14, 13), n_ply=7, nparts=(2, 1, 1), nev=8),
    "lam_wide17": lambda: gen.small_case("laminate", seed=33, nxy=(14, 20), n_ply=11, nparts=(2, 1, 1), nev=8),
    "lam_wide22": lambda: gen.small_case("laminate", seed=34, nxy=(22, 17), n_ply=9, nparts=(2, 1, 1), nev=8),
}


# Variants of a case: name + "|" + comma-separated field=value pairs of the
# workload (overlap=2, pou=sarkis), e.g. "lam_3x2x2_uneven|overlap=2,pou=sarkis".
@functools.lru_cache(maxsize=None)
def workload(name):
    base, _, mods = name.partition("|")
    w = (CASES.get(base) or WIDE[base])()
    if mods:
        kw = {}
        for item in mods.split(","):
            k, v = item.split("=")
            kw[k] = int(v) if v.isdigit() else v
        w = dataclasses.replace(w, **kw)
    return w


def _n_eig(name):
    """Eigenpairs the oracle computes per subdomain: all for the small cases,
    the smallest (nev or nev_max) + 12 for the wide ones."""
    if name.partition("|")[0] in CASES:
        return None
    w = workload(name)
    return max(w.nev, w.nev_max) + 12


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
    return geneo.GenEO(w, A, Ke, coarse=coarse, keep_all=True, n_eig=_n_eig(name) if coarse else None)


def eta_vectors(n):
    """Fixed random vectors on which two implementations' operators are compared."""
    return np.random.default_rng(5).standard_normal((4, n))


def operator_eta(A, X, AX):
    """Normwise relative difference of another implementation's products AX
    (rows of AX = A X_i) from this operator:
    max_i ||AX_i - A X_i||_2 / || |A| |X_i| ||_2."""
    absA = abs(A)
    return max(float(np.linalg.norm(AX[i] - A @ X[i]) / np.linalg.norm(absA @ np.abs(X[i])))
               for i in range(X.shape[0]))


@functools.lru_cache(maxsize=None)
def minv_sensitivity(name, coarse=True, seed=3):
    """FP64 condition of M^-1 r on this case: the largest relative change of the
    oracle's M^-1 r (r standard normal, the given seed) when every element
    matrix is perturbed by independent relative rounding-size noise
    (K_e (1 + eps xi), symmetrised; two draws) and A, the local factors, the
    pencils, the coarse space and A_H are all rebuilt from it.  Returns
    dict(s=that change, eta=the operator_eta of the perturbed operators, the
    size of the perturbation in the normwise measure)."""
    w = workload(name)
    A, b, free, Ke = system(name)
    ref_run = geneo_run(name, coarse)
    r = np.random.default_rng(seed).standard_normal(w.n_free)
    ref = ref_run.apply(r)
    X = eta_vectors(w.n_free)
    worst = eta = 0.0
    for s in (11, 12):
        xi = np.random.default_rng(s).standard_normal(Ke.shape)
        Kp = Ke * (1.0 + np.finfo(float).eps * xi)
        Kp = 0.5 * (Kp + np.transpose(Kp, (0, 2, 1)))
        Ap, bp, fp = fem.assemble(w, Kp)
        eta = max(eta, operator_eta(A, X, np.stack([Ap @ x for x in X])))
        gp_ = geneo.GenEO(w, Ap, Kp, coarse=coarse, n_eig=_n_eig(name) if coarse else None)
        worst = max(worst, float(np.linalg.norm(gp_.apply(r) - ref) / np.linalg.norm(ref)))
    return dict(s=worst, eta=eta)


def minv_eps_sensitivity(name, coarse=True, seed=3):
    return minv_sensitivity(name, coarse, seed)["s"]


def minv_gate(name, coarse=True, seed=3, eta=None):
    """Relative tolerance for M^-1 r against the oracle: 1e-10, or three times
    the case's FP64 condition (minv_sensitivity) where that is larger.  Two FP64
    implementations round their element integrals differently, so their
    operators differ by some eta (operator_eta; the assembly parity test bounds
    it by 32 eps): given the other implementation's measured eta, the condition,
    measured for a perturbation of size sens["eta"], is scaled linearly to it
    (first-order perturbation theory), never below the unscaled value."""
    sens = minv_sensitivity(name, coarse, seed)
    scale = max(1.0, eta / sens["eta"]) if eta is not None and sens["eta"] > 0 else 1.0
    return max(1e-10, 3.0 * sens["s"] * scale)


def check_eigenvalues(w, g, eig_of):
    """GenEO eigenvalues and counts against the oracle (Section 3.2, eq-geneo).

    m_j equal; the first m_j + 1 eigenvalues agree to
    1e-10 max(|lambda_ref|, 1e-3 lambda_cut), lambda_cut = the threshold (or
    lambda_m for a fixed count): relative 1e-10 except far below the cut, where
    only an absolute accuracy relative to the cut is meaningful.  Exact zeros
    (rigid-body or constant modes of floating subdomains) carry only rounding:
    both sides must put them below 1e-9 lambda_{m+1}."""
    for j in range(w.n_sub):
        lam, m = eig_of(j)
        lref = g.lam[j]
        assert m == g.m[j], (j, m, g.m[j], lam[:m + 2], lref[:m + 2])
        k = m + 1
        zero = 1e-9 * abs(lref[m])
        z = np.abs(lref[:k]) < zero
        assert np.all(np.abs(lam[:k][z]) < zero), (j, lam[:k], lref[:k])
        lam_cut = w.threshold if w.nev <= 0 else abs(lref[m - 1])
        tol = 1e-10 * np.maximum(np.abs(lref[:k]), 1e-3 * lam_cut)
        err = np.abs(lam[:k] - lref[:k])
        assert np.all(err[~z] <= tol[~z]), (j, lam[:k], lref[:k], err, tol)


@functools.lru_cache(maxsize=None)
def pcg_run(name, rtol=1e-12):
    A, b, free, Ke = system(name)
    g = geneo_run(name)
    return pcg.pcg(A, b[:, 0], g.apply, rtol=rtol, maxit=2000)
