"""Oracle: GenEO local eigenproblems, coarse space and coarse matrix.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 3.1 defines the local Dirichlet matrices A_j = R_j A R_j^T.  Section
3.2 (eq-geneo) defines, on each subdomain, the generalised eigenproblem
a_{Omega_j}(p, v) = lambda a_{Omega_j^o}(Xi_j p, Xi_j v) for all v in
V_h(Omega_j); Section 3.3.2 (eqm:matrixForm) writes it as
A_{Omega_j} p = lambda X A_{Omega_j^o} X p with ascending eigenvalues and
||p||_2 = 1, solved in shift-and-invert mode with a small shift.  The GenEO
coarse space (its Definition in Section 3.2) is spanned by R_j^T Xi_j p_k^j,
k <= m_j; Section 3.3.2 numbers the basis Phi_{i(j,k)} = X^(j) p_k^j padded by
zeros, N_H = sum_j m_j; Section 3.3.3 defines A_H = R_H A R_H^T.

The oracle computes the eigenpairs with dense linear algebra: with
P = A_N + s B (SPD for s > 0) and its Cholesky factor L, the pencil is
equivalent to the symmetric problem  L^-1 B L^-T w = nu w  with
lambda = 1/nu - s and p = L^-T w; each finite eigenvalue is then reported as
the Rayleigh quotient p^T A_N p / p^T B p of its eigenvector, which does not
lose the digits that 1/nu - s cancels when lambda is far below s.  A_H is formed from its global definition
Phi^T (A Phi), not from the local products the GPU uses.

Readings: the shift is s = 1e-2 (algorithmic only: the eigenvalues do not
depend on it, and a test runs two shifts); m_j is either a fixed count or the
number of eigenvalues strictly below a threshold (capped), then extended while
the next eigenvalue is equal to the last within 1e-8 relative (+1e-10
absolute) so that a degenerate cluster is never split; each eigenvector is
scaled to unit 2-norm with its largest-magnitude entry positive (lowest index
on ties).

The zero-energy-mode (ZEM) coarse space the paper compares against (Section 5,
Example 1b: no coarse space, only the zero energy modes, or GenEO) takes on
each subdomain the kernel of its Neumann matrix A_{Omega_j}: the constant
(scalar diffusion) or the six rigid-body translations and rotations
(elasticity).  Reading: only floating subdomains, whose elements touch no
Dirichlet DOF, contribute (a subdomain meeting a clamped face has no kernel);
this is also what the coarse dimensions of the paper's Example 1b table
count (six per subdomain off the clamped end).  Its basis is X_j z_k like the
GenEO one.

Pins (tests/test_oracle_geneo.py): eigen residual ||A_N p - lambda B p||,
B-orthogonality, exactly 6 (elasticity) / 1 (scalar) zero eigenvalues on
floating subdomains and none on clamped ones, independence of the shift, a
brute-force characteristic-polynomial check on a tiny pencil, A_H by local
products equal to the global product, A_H SPD.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import fem
from .dd import Decomposition
from .fem import elem_dofs


def local_dirichlet(A, I) -> np.ndarray:
    """A_j = R_j A R_j^T as a dense matrix (Section 3.1)."""
    return A[I][:, I].toarray()


def local_assembly(w, dec: Decomposition, Ke: np.ndarray, j: int, elem_mask: np.ndarray,
                   dofs_local: np.ndarray) -> np.ndarray:
    """Sum of K_e over the masked elements on the DOF list ``dofs_local`` (free ids)."""
    pos = -np.ones(w.n_free, dtype=np.int64)
    pos[dofs_local] = np.arange(len(dofs_local))
    n = len(dofs_local)
    M = np.zeros((n, n))
    el = np.flatnonzero(elem_mask)
    fd = dec.free_of_full[elem_dofs(w, dec.en[el])]
    for t in range(len(el)):
        f = fd[t]
        keep = f >= 0
        loc = pos[f[keep]]
        if np.any(loc < 0):
            raise ValueError("element DOF outside the local DOF set")
        M[np.ix_(loc, loc)] += Ke[el[t]][np.ix_(keep, keep)]
    return M


def pencil(w, dec: Decomposition, Ke: np.ndarray, j: int):
    """(A_N, B) on Ibar_j: A_N = A_{Omega_j}, B = X A_{Omega_j^o} X."""
    Ib = dec.Ibar[j]
    AN = local_assembly(w, dec, Ke, j, dec.E[j], Ib)
    AO = local_assembly(w, dec, Ke, j, dec.E_ov[j], Ib)
    X = dec.X[j]
    B = X[:, None] * AO * X[None, :]
    return AN, B


def pencil_eig(AN: np.ndarray, B: np.ndarray, shift: float = 1e-2, n_eig: int | None = None):
    """All eigenpairs (ascending lambda, inf for the null space of B), or only
    the n_eig smallest when n_eig is given."""
    P = AN + shift * B
    L = np.linalg.cholesky(P)
    Linv_B = sla.solve_triangular(L, B, lower=True)
    C = sla.solve_triangular(L, Linv_B.T, lower=True)    # L^-1 B L^-T (symmetric)
    C = 0.5 * (C + C.T)
    n = C.shape[0]
    if n_eig is not None and n_eig < n:
        nu, W = sla.eigh(C, subset_by_index=[n - n_eig, n - 1])
    else:
        nu, W = np.linalg.eigh(C)
    order = np.argsort(-nu)                                # largest nu first
    nu, W = nu[order], W[:, order]
    with np.errstate(divide="ignore"):
        lam = np.where(nu > 1e-14 / shift, 1.0 / nu - shift, np.inf)
    Pv = sla.solve_triangular(L.T, W, lower=False)
    Pv = normalise(Pv)
    # Each finite eigenvalue is reported as the Rayleigh quotient of its own
    # pencil, p^T A_N p / p^T B p (eq-geneo with v = p).  Forming 1/nu - s
    # subtracts two numbers near 1/s when lambda << s and loses about
    # log10(s / lambda) digits; the quotient of the two energies does not.
    fin = np.isfinite(lam)
    if np.any(fin):
        Pf = Pv[:, fin]
        lam = lam.copy()
        lam[fin] = np.einsum("ik,ik->k", Pf, AN @ Pf) / np.einsum("ik,ik->k", Pf, B @ Pf)
    return lam, Pv


def normalise(Pv: np.ndarray) -> np.ndarray:
    """Unit 2-norm columns, largest-magnitude entry positive (first on ties)."""
    Pv = Pv / np.linalg.norm(Pv, axis=0, keepdims=True)
    idx = np.argmax(np.abs(Pv), axis=0)
    sgn = np.sign(Pv[idx, np.arange(Pv.shape[1])])
    sgn[sgn == 0] = 1.0
    return Pv * sgn[None, :]


def zem_basis(w, dec: Decomposition, j: int) -> np.ndarray:
    """Zero-energy modes on Ibar_j (columns, unit 2-norm): the constant for the
    scalar problem, the three translations and three infinitesimal rotations
    u = theta x (x - c) about the box centre c for elasticity; an empty basis
    when the subdomain's nodes carry a Dirichlet DOF."""
    nc = w.ncomp
    nodes = np.unique(dec.en[dec.E[j]].ravel())
    dofs_all = (nodes[:, None] * nc + np.arange(nc)[None, :]).ravel()
    Ib = dec.Ibar[j]
    if np.any(w.dirichlet[dofs_all] != 0):
        return np.zeros((len(Ib), 0))
    full = w.free_index()[Ib]
    node, comp = full // nc, full % nc
    if nc == 1:
        Z = np.ones((len(Ib), 1))
    else:
        X = fem.node_xyz(w)[node]
        allx = fem.node_xyz(w)[nodes]
        c = 0.5 * (allx.min(axis=0) + allx.max(axis=0))
        d = X - c
        Z = np.zeros((len(Ib), 6))
        for a in range(3):
            Z[:, a] = (comp == a)
        # rotations about x, y, z: theta_a e_a x d
        for a in range(3):
            th = np.zeros(3)
            th[a] = 1.0
            u = np.cross(th[None, :], d)
            Z[:, 3 + a] = u[np.arange(len(Ib)), comp]
    return Z / np.linalg.norm(Z, axis=0, keepdims=True)


def select_count(lam: np.ndarray, nev: int, threshold: float, nev_max: int) -> int:
    """m_j: fixed count, or #{lambda < threshold} capped; then cluster completion."""
    finite = int(np.sum(np.isfinite(lam)))
    if nev > 0:
        m = min(nev, finite)
    else:
        m = int(np.sum(lam < threshold))
        if nev_max > 0:
            m = min(m, nev_max)
    cap = nev_max if nev_max > 0 else finite
    cap = max(cap, m)
    while 0 < m < min(cap, finite) and lam[m] - lam[m - 1] <= 1e-8 * abs(lam[m - 1]) + 1e-10:
        m += 1
    return m


class GenEO:
    """Local factors, eigenpairs, coarse basis and coarse matrix."""

    def __init__(self, w, A, Ke, dec: Decomposition | None = None, shift: float = 1e-2,
                 coarse=True, keep_all: bool = False, coarse_solve: str = "exact",
                 coarse_rtol: float = 1e-4, coarse_maxit: int = 200, n_eig: int | None = None):
        """coarse: True (or "geneo") for the GenEO coarse space, "zem" for the
        zero-energy modes of floating subdomains, False for one level only.
        coarse_solve: "exact" (Cholesky of A_H) or "cg" (inexact: conjugate
        gradients on A_H preconditioned by the inverses of its diagonal blocks,
        one block per subdomain, x0 = 0, stopped at coarse_rtol relative
        residual or coarse_maxit iterations; Section 3.3.3, last paragraph).
        n_eig: compute only that many of the smallest eigenpairs per subdomain
        (large subdomains); the count selected must stay below it."""
        self.coarse_solve = coarse_solve
        self.coarse_rtol, self.coarse_maxit = coarse_rtol, coarse_maxit
        self.coarse_iters = []
        self.w = w
        self.A = A
        self.dec = dec if dec is not None else Decomposition(w)
        self.shift = shift
        d = self.dec
        self.Aj_chol = []
        for I in d.I:
            self.Aj_chol.append(sla.cho_factor(local_dirichlet(A, I), lower=True))
        self.lam, self.m, self.P = [], [], []
        if not coarse:
            self.NH = 0
            return
        for j in range(d.n_sub):
            if coarse == "zem":
                Zj = zem_basis(w, d, j)
                self.m.append(Zj.shape[1])
                self.P.append(Zj)
                continue
            AN, B = pencil(w, d, Ke, j)
            lam, Pv = pencil_eig(AN, B, shift, n_eig)
            m = select_count(lam, w.nev, w.threshold, w.nev_max)
            if n_eig is not None and m >= len(lam) - 1:
                raise ValueError("n_eig too small for the selected eigenvectors")
            self.lam.append(lam if keep_all else lam[: max(m + 8, 16)])
            self.m.append(m)
            self.P.append(Pv[:, :m])
        self.offsets = np.concatenate([[0], np.cumsum(self.m)]).astype(np.int64)
        self.NH = int(self.offsets[-1])
        Phi = np.zeros((w.n_free, self.NH))
        for j in range(d.n_sub):
            Ib = d.Ibar[j]
            Phi[Ib, self.offsets[j]: self.offsets[j + 1]] = d.X[j][:, None] * self.P[j]
        self.Phi = Phi
        self.AH = Phi.T @ (A @ Phi)
        self.AH = 0.5 * (self.AH + self.AH.T)
        self.AH_chol = sla.cho_factor(self.AH, lower=True) if self.NH > 0 else None
        # diagonal blocks of A_H (one per subdomain) for the inexact coarse solve
        self.AH_dinv = [np.linalg.inv(self.AH[a:c, a:c]) if c > a else np.zeros((0, 0))
                        for a, c in zip(self.offsets[:-1], self.offsets[1:])]

    def coarse_cg(self, g: np.ndarray) -> np.ndarray:
        """Inexact A_H^-1 g: preconditioned CG on A_H, block-Jacobi M^-1 = blockdiag(A_jj)^-1."""
        def prec(v):
            out = np.zeros_like(v)
            for j, Dj in enumerate(self.AH_dinv):
                a, c = self.offsets[j], self.offsets[j + 1]
                out[a:c] = Dj @ v[a:c]
            return out
        y, info = _inner_pcg(self.AH, g, prec, self.coarse_rtol, self.coarse_maxit)
        self.coarse_iters.append(info)
        return y

    def apply_as1(self, r: np.ndarray) -> np.ndarray:
        """One-level additive Schwarz sum_j R_j^T A_j^-1 R_j r (eqn:onelevelAS)."""
        z = np.zeros_like(r)
        for I, c in zip(self.dec.I, self.Aj_chol):
            z[I] += sla.cho_solve(c, r[I])
        return z

    def apply_coarse(self, r: np.ndarray) -> np.ndarray:
        """R_H^T A_H^-1 R_H r with (R_H v)_i = Phi_i^T v (Section 3.3.3)."""
        if self.NH == 0:
            return np.zeros_like(r)
        g = self.Phi.T @ r
        y = self.coarse_cg(g) if self.coarse_solve == "cg" else sla.cho_solve(self.AH_chol, g)
        return self.Phi @ y

    def apply(self, r: np.ndarray) -> np.ndarray:
        """Two-level additive Schwarz M^-1_{AS,2} r (Section 3.1)."""
        return self.apply_as1(r) + self.apply_coarse(r)


def _inner_pcg(AH, g, prec, rtol, maxit):
    """Plain PCG for the coarse system, x0 = 0, stop at ||r|| <= rtol ||g||."""
    y = np.zeros_like(g)
    r = g.copy()
    ng = np.linalg.norm(g)
    if ng == 0.0:
        return y, 0
    z = prec(r)
    p = z.copy()
    rz = r @ z
    k = 0
    while k < maxit:
        q = AH @ p
        a = rz / (p @ q)
        y += a * p
        r -= a * q
        k += 1
        if np.linalg.norm(r) <= rtol * ng:
            break
        z = prec(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return y, k
