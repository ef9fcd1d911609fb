"""Oracle: preconditioned conjugate gradients and the CG-Lanczos estimate.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 3.1: CG (Hestenes-Stiefel) builds iterates in the Krylov space
eqn:KrylovSubspace, with search directions A-orthogonal to the previous ones,
until the residual norm falls below a user tolerance; the preconditioned
system M^-1 A u = M^-1 b uses M^-1 = M^-1_{AS,1} (eqn:onelevelAS) or
M^-1_{AS,2} (two-level additive Schwarz).  The tables report a condition
number estimate of M^-1 A; the reading here is the extreme eigenvalues of the
Lanczos tridiagonal built from the CG coefficients.

Readings: x0 = 0; stop when ||r_k||_2 <= rtol ||b||_2 (unpreconditioned
residual); the true residual b - A x is recomputed at exit.  The paper's
flexible Krylov method for an inexact coarse solve is FGMRES; here the
flexible variant of CG (Polak-Ribiere beta) takes its place, so that one
short-recurrence loop serves both cases.

Pins (tests/test_oracle_pcg.py): dense direct solve on tiny meshes, one
subdomain => one iteration, symmetry of M^-1, kappa estimate against the
dense spectrum of M^-1 A.
"""
from __future__ import annotations

import numpy as np


def pcg(A, b: np.ndarray, Minv=None, rtol: float = 1e-8, maxit: int = 1000, flexible: bool = False):
    """Returns (x, info) with iterations, histories, alpha/beta and residuals.

    flexible=True takes the Polak-Ribiere form of beta,
    beta = z_{k+1}^T (r_{k+1} - r_k) / z_k^T r_k, which equals the standard one
    when M^-1 is a fixed symmetric operator (then z_{k+1}^T r_k = 0) and keeps
    CG converging when M^-1 changes from one application to the next (an
    inexact coarse solve, Section 3.3.3 last paragraph, where the paper switches
    to a flexible Krylov method)."""
    n = b.shape[0]
    x = np.zeros(n)
    r = b.copy()
    nb = np.linalg.norm(b)
    info = dict(iters=0, res=[np.linalg.norm(r) / nb if nb > 0 else 0.0], alpha=[], beta=[],
                converged=False)
    if nb == 0.0:
        info["converged"] = True
        info["true_rel_res"] = 0.0
        return x, info
    z = Minv(r) if Minv is not None else r.copy()
    p = z.copy()
    rz = r @ z
    for k in range(maxit):
        q = A @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r_old = r.copy()
        r -= alpha * q
        info["alpha"].append(alpha)
        info["iters"] = k + 1
        rel = np.linalg.norm(r) / nb
        info["res"].append(rel)
        if rel <= rtol:
            info["converged"] = True
            break
        z = Minv(r) if Minv is not None else r.copy()
        rz_new = r @ z
        beta = (z @ (r - r_old)) / rz if flexible else rz_new / rz
        info["beta"].append(beta)
        p = z + beta * p
        rz = rz_new
    info["true_rel_res"] = float(np.linalg.norm(b - A @ x) / nb)
    info["kappa"] = kappa_estimate(info["alpha"], info["beta"])
    return x, info


def lanczos_tridiagonal(alpha, beta) -> np.ndarray:
    """T_k of the preconditioned operator from CG coefficients:
    T_ii = 1/alpha_i + beta_{i-1}/alpha_{i-1},  T_{i,i+1} = sqrt(beta_i)/alpha_i."""
    k = len(alpha)
    T = np.zeros((k, k))
    for i in range(k):
        T[i, i] = 1.0 / alpha[i] + (beta[i - 1] / alpha[i - 1] if i > 0 else 0.0)
        if i + 1 < k:
            T[i, i + 1] = T[i + 1, i] = np.sqrt(beta[i]) / alpha[i]
    return T


def kappa_estimate(alpha, beta) -> float:
    if len(alpha) == 0:
        return 1.0
    ev = np.linalg.eigvalsh(lanczos_tridiagonal(alpha, beta))
    return float(ev[-1] / ev[0])
