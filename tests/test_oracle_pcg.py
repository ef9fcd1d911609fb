"""Pins of the oracle's PCG, preconditioners and condition estimate (Section 3.1)."""
import numpy as np
import pytest

from oracle import dd, fem, geneo, pcg
from workloads import generate as gen


def _setup(kind, seed=0, **kw):
    w = gen.small_case(kind, seed=seed, **kw)
    A, b, free = fem.assemble(w)
    Ke = fem.element_matrices(w)
    return w, A, b, Ke


@pytest.mark.parametrize("kind,kw", [
    ("laminate", dict(nxy=(6, 4), n_ply=2, nparts=(2, 2, 1), nev=6)),
    ("diffusion", dict(ne=(8, 6, 5), nparts=(2, 2, 1), threshold=0.2, nev_max=8)),
])
def test_pcg_matches_dense_direct_solve(kind, kw):
    w, A, b, Ke = _setup(kind, seed=1, **kw)
    u_ref = np.linalg.solve(A.toarray(), b[:, 0])
    g = geneo.GenEO(w, A, Ke)
    u, info = pcg.pcg(A, b[:, 0], g.apply, rtol=1e-13, maxit=500)
    assert info["converged"]
    assert np.linalg.norm(u - u_ref) <= 1e-10 * np.linalg.norm(u_ref)
    # attainable true residual is ~ eps * ||A|| ||u|| / ||b|| (thin resin layers make A ill-conditioned)
    assert info["true_rel_res"] <= 1e-9


def test_single_subdomain_is_exact_inverse():
    w, A, b, Ke = _setup("laminate", seed=2, nxy=(5, 4), n_ply=2, nparts=(1, 1, 1), nev=0,
                         threshold=0.0)
    g = geneo.GenEO(w, A, Ke, coarse=False)
    u, info = pcg.pcg(A, b[:, 0], g.apply, rtol=1e-10)
    assert info["iters"] == 1


@pytest.mark.parametrize("coarse", [False, True])
def test_preconditioner_symmetric_positive_definite(coarse):
    w, A, b, Ke = _setup("laminate", seed=3, nxy=(6, 4), n_ply=2, nparts=(3, 2, 1), nev=4)
    g = geneo.GenEO(w, A, Ke, coarse=coarse)
    n = w.n_free
    M = np.stack([g.apply(e) for e in np.eye(n)], axis=1)
    assert np.max(np.abs(M - M.T)) <= 1e-10 * np.max(np.abs(M))
    assert np.linalg.eigvalsh(0.5 * (M + M.T))[0] > 0


def test_kappa_estimate_against_dense_spectrum():
    w, A, b, Ke = _setup("laminate", seed=4, nxy=(6, 4), n_ply=2, nparts=(2, 2, 1), nev=4)
    g = geneo.GenEO(w, A, Ke)
    n = w.n_free
    M = np.stack([g.apply(e) for e in np.eye(n)], axis=1)
    ev = np.sort(np.linalg.eigvals(M @ A.toarray()).real)
    kappa = ev[-1] / ev[0]
    rhs = np.random.default_rng(0).standard_normal(n)
    _, info = pcg.pcg(A, rhs, g.apply, rtol=1e-14, maxit=400)
    assert abs(info["kappa"] - kappa) <= 1e-3 * kappa


def test_geneo_flat_where_one_level_grows():
    # qualitative Table 1 pattern: more subdomains -> one-level AS condition number
    # and iterations grow, while the GenEO estimate stays O(10)
    it_as, it_g, k_as, k_g = [], [], [], []
    for nparts in [(2, 1, 1), (8, 2, 1)]:
        w, A, b, Ke = _setup("laminate", seed=5, nxy=(16, 4), n_ply=3, nparts=nparts, nev=8)
        g = geneo.GenEO(w, A, Ke)
        _, i1 = pcg.pcg(A, b[:, 0], g.apply_as1, rtol=1e-8, maxit=2000)
        _, i2 = pcg.pcg(A, b[:, 0], g.apply, rtol=1e-8, maxit=2000)
        it_as.append(i1["iters"])
        it_g.append(i2["iters"])
        k_as.append(i1["kappa"])
        k_g.append(i2["kappa"])
    assert it_as[1] > 2 * it_as[0] and k_as[1] > 10 * k_as[0]
    assert max(k_g) < 20
    assert it_g[1] < it_as[1] / 2


def test_flexible_cg_with_exact_preconditioner_reproduces_pcg():
    """Polak-Ribiere beta equals the standard beta when M^-1 is fixed and
    symmetric: the same iterates up to rounding, the same iteration count."""
    w, A, b, Ke = _setup("laminate", seed=8, nxy=(8, 6), n_ply=2, nparts=(2, 2, 1), nev=6)
    g = geneo.GenEO(w, A, Ke)
    u1, i1 = pcg.pcg(A, b[:, 0], g.apply, rtol=1e-10, maxit=500)
    u2, i2 = pcg.pcg(A, b[:, 0], g.apply, rtol=1e-10, maxit=500, flexible=True)
    assert abs(i1["iters"] - i2["iters"]) <= 1
    assert np.linalg.norm(u1 - u2) <= 1e-8 * np.linalg.norm(u1)
    assert np.allclose(i1["alpha"][:10], i2["alpha"][:10], rtol=1e-6)


@pytest.mark.parametrize("kind,kw", [
    ("laminate", dict(nxy=(12, 6), n_ply=2, nparts=(3, 2, 1), nev=6)),
    ("diffusion", dict(ne=(12, 10, 6), nparts=(3, 2, 1), threshold=0.2, nev_max=8)),
])
def test_inexact_coarse_solve_with_flexible_cg_converges_to_the_solution(kind, kw):
    """Section 3.3.3, last paragraph: with the coarse system solved iteratively
    (CG on A_H with block-Jacobi, here stopped at a loose 1e-1) the
    preconditioner changes from one application to the next; flexible CG still
    converges to A^-1 b and needs no more iterations than the standard
    recurrence with the same inexact preconditioner (on the laminate, whose
    A_H is ill-conditioned, far fewer).  A tight inner tolerance reproduces the
    exact coarse correction."""
    w, A, b, Ke = _setup(kind, seed=9, **kw)
    u_ref = np.linalg.solve(A.toarray(), b[:, 0])
    ex = geneo.GenEO(w, A, Ke)
    ue, ie = pcg.pcg(A, b[:, 0], ex.apply, rtol=1e-10, maxit=500)
    inx = geneo.GenEO(w, A, Ke, coarse_solve="cg", coarse_rtol=1e-1, coarse_maxit=200)
    uf, fi = pcg.pcg(A, b[:, 0], inx.apply, rtol=1e-10, maxit=1000, flexible=True)
    assert fi["converged"]
    assert np.linalg.norm(uf - u_ref) <= 1e-8 * np.linalg.norm(u_ref)
    assert fi["iters"] <= 2 * ie["iters"]
    std = geneo.GenEO(w, A, Ke, coarse_solve="cg", coarse_rtol=1e-1, coarse_maxit=200)
    us, si = pcg.pcg(A, b[:, 0], std.apply, rtol=1e-10, maxit=1000)
    assert fi["iters"] <= si["iters"]
    if kind == "laminate":
        assert 2 * fi["iters"] < si["iters"], (fi["iters"], si["iters"])
        assert max(inx.coarse_iters) >= 2      # the inner solve really is iterative
    r = np.random.default_rng(0).standard_normal(w.n_free)
    tight = geneo.GenEO(w, A, Ke, coarse_solve="cg", coarse_rtol=1e-13, coarse_maxit=2000)
    assert np.linalg.norm(tight.apply(r) - ex.apply(r)) <= 1e-9 * np.linalg.norm(ex.apply(r))
