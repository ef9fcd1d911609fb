"""Pins of the oracle's GenEO eigenproblems and coarse space (Sections 3.2, 3.3)."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import dd, fem, geneo
from workloads import generate as gen


def _setup(kind, seed=0, **kw):
    w = gen.small_case(kind, seed=seed, **kw)
    A, b, free = fem.assemble(w)
    Ke = fem.element_matrices(w)
    d = dd.Decomposition(w)
    return w, A, b, Ke, d


def test_known_spectrum_pencil():
    # A = V^-T Da V^-1, B = V^-T Db V^-1 has eigenvalues Da/Db (inf where Db = 0)
    rng = np.random.default_rng(3)
    n = 9
    V = rng.standard_normal((n, n)) + 3 * np.eye(n)
    Vi = np.linalg.inv(V)
    Da = np.array([0.0, 0.0, 0.3, 1.0, 2.0, 5.0, 7.0, 1.0, 4.0])
    Db = np.array([1.0, 2.0, 1.0, 0.5, 1.0, 1.0, 0.0, 0.0, 2.0])
    A = Vi.T @ np.diag(Da + 1e-300) @ Vi
    A = A + Vi.T @ np.diag((Db == 0) * 3.0) @ Vi   # keep A + sB definite on null(B)
    B = Vi.T @ np.diag(Db) @ Vi
    A, B = 0.5 * (A + A.T), 0.5 * (B + B.T)
    lam, P = geneo.pencil_eig(A, B, shift=1e-2)
    expect = np.sort(np.where(Db > 0, Da / np.where(Db > 0, Db, 1), np.inf))
    fin = np.isfinite(expect)
    assert np.allclose(lam[fin], expect[fin], atol=1e-10)
    assert np.all(~np.isfinite(lam[~fin]) | (lam[~fin] > 1e8))


@pytest.mark.parametrize("kind,kw,zero_modes", [
    ("laminate", dict(nxy=(8, 6), n_ply=2, nparts=(2, 2, 1)), 6),
    ("diffusion", dict(ne=(10, 8, 6), nparts=(2, 2, 2), dirichlet_faces=("x0",)), 1),
])
def test_eigen_residual_zero_modes_and_shift_independence(kind, kw, zero_modes):
    w, A, b, Ke, d = _setup(kind, seed=4, **kw)
    boxes = dd.subdomain_boxes(w)
    for j in range(d.n_sub):
        AN, B = geneo.pencil(w, d, Ke, j)
        lam, P = geneo.pencil_eig(AN, B, 1e-2)
        k = 12
        nA = np.linalg.norm(AN, 2)
        for i in range(k):
            r = AN @ P[:, i] - lam[i] * (B @ P[:, i])
            assert np.linalg.norm(r) <= 1e-10 * nA, (j, i)
        G = P[:, :k].T @ B @ P[:, :k]
        off = G - np.diag(np.diag(G))
        assert np.max(np.abs(off)) <= 1e-9 * np.max(np.abs(np.diag(G)))
        floating = boxes[j][0][0] > 0           # not touching the Dirichlet face x = 0
        nzero = int(np.sum(np.abs(lam) < 1e-8))
        assert nzero == (zero_modes if floating else 0), (j, lam[:8])
        lam2, _ = geneo.pencil_eig(AN, B, 1e-1)
        sel = lam[:k] > 1e-6
        assert np.allclose(lam2[:k][sel], lam[:k][sel], rtol=1e-10, atol=0)


def test_selection_rule_and_cluster_completion():
    lam = np.array([0.0, 0.0, 0.01, 0.05, 0.05 * (1 + 1e-12), 0.2, np.inf])
    assert geneo.select_count(lam, 4, 0, 0) == 5          # cluster completed
    assert geneo.select_count(lam, 2, 0, 0) == 2
    assert geneo.select_count(lam, 0, 0.15, 0) == 5
    assert geneo.select_count(lam, 0, 0.15, 3) == 3
    assert geneo.select_count(lam, 0, 0.3, 0) == 6


def test_local_dirichlet_matrix_equals_local_assembly():
    w, A, b, Ke, d = _setup("laminate", seed=2, nxy=(8, 6), n_ply=2, nparts=(2, 2, 1))
    for j in range(d.n_sub):
        Aj = geneo.local_dirichlet(A, d.I[j])
        loc = geneo.local_assembly(w, d, Ke, j, d.E[j], d.Ibar[j])
        pos = np.searchsorted(d.Ibar[j], d.I[j])
        assert np.allclose(Aj, loc[np.ix_(pos, pos)], rtol=0, atol=1e-9 * abs(Aj).max())


@pytest.mark.parametrize("kind,kw", [
    ("laminate", dict(nxy=(8, 6), n_ply=2, nparts=(2, 2, 1), nev=6)),
    ("diffusion", dict(ne=(10, 8, 6), nparts=(2, 2, 2), threshold=0.3, nev_max=10)),
])
def test_coarse_matrix_local_products_equal_global(kind, kw):
    w, A, b, Ke, d = _setup(kind, seed=3, **kw)
    g = geneo.GenEO(w, A, Ke, d)
    assert g.NH == sum(g.m) and g.NH > 0
    # Section 3.3.3: (A_H)_{il} = Phi_i^T  Atilde_{j(i)} Phi_l with Atilde_j = A on Ibar_j
    AH = np.zeros((g.NH, g.NH))
    for j in range(d.n_sub):
        Ib = d.Ibar[j]
        At = A[Ib][:, Ib]
        rows = slice(g.offsets[j], g.offsets[j + 1])
        AH[rows, :] = g.Phi[Ib, rows].T @ (At @ g.Phi[Ib, :])
    assert np.allclose(AH, g.AH, rtol=0, atol=1e-10 * np.abs(g.AH).max())
    ev = np.linalg.eigvalsh(g.AH)
    assert ev[0] > 0


def test_coarse_correction_invariant_under_basis_change():
    w, A, b, Ke, d = _setup("laminate", seed=3, nxy=(8, 6), n_ply=2, nparts=(2, 2, 1), nev=5)
    g = geneo.GenEO(w, A, Ke, d)
    r = np.random.default_rng(1).standard_normal(w.n_free)
    z1 = g.apply_coarse(r)
    Gm = np.random.default_rng(2).standard_normal((g.NH, g.NH)) + 4 * np.eye(g.NH)
    Phi2 = g.Phi @ Gm
    AH2 = Phi2.T @ (A @ Phi2)
    z2 = Phi2 @ np.linalg.solve(AH2, Phi2.T @ r)
    assert np.allclose(z1, z2, rtol=1e-8, atol=1e-10 * np.abs(z1).max())


@pytest.mark.parametrize("kind,kw,nmodes", [
    ("laminate", dict(nxy=(8, 6), n_ply=2, nparts=(2, 2, 1)), 6),
    ("laminate", dict(nxy=(10, 4), n_ply=2, nparts=(3, 1, 1), ramp=(3.0, 7.0, 0.17)), 6),
    ("diffusion", dict(ne=(10, 8, 6), nparts=(2, 2, 2), dirichlet_faces=("x0",)), 1),
])
def test_zem_basis_is_the_neumann_kernel(kind, kw, nmodes):
    """The zero-energy modes span exactly the kernel of A_{Omega_j}: A_N Z = 0,
    full rank, the same span as the pencil's zero eigenvalues, and present only
    on subdomains that do not touch the Dirichlet face."""
    w, A, b, Ke, d = _setup(kind, seed=5, **kw)
    boxes = dd.subdomain_boxes(w)
    for j in range(d.n_sub):
        Z = geneo.zem_basis(w, d, j)
        floating = boxes[j][0][0] > 0
        assert Z.shape[1] == (nmodes if floating else 0), j
        if not floating:
            continue
        AN, B = geneo.pencil(w, d, Ke, j)
        assert np.linalg.norm(AN @ Z) <= 1e-10 * np.linalg.norm(AN, 2) * np.linalg.norm(Z, 2)
        sv = np.linalg.svd(Z, compute_uv=False)
        assert sv[-1] >= 1e-3 * sv[0]
        lam, P = geneo.pencil_eig(AN, B, 1e-2)
        Q, _ = np.linalg.qr(P[:, np.abs(lam) < 1e-8])
        assert Q.shape[1] == nmodes
        assert np.linalg.norm(Z - Q @ (Q.T @ Z)) <= 1e-8 * np.linalg.norm(Z)


def test_coarse_spaces_order_like_the_example_1b_table():
    """One level, ZEM and GenEO on a clamped laminate split along x: the ZEM
    coarse dimension is six per subdomain off the clamped end, and the
    iterations to a 1e-5 residual reduction fall AS > ZEM > GenEO (the pattern
    of the paper's Example 1b table; exact counts are not pinned)."""
    from oracle import pcg
    w = gen.small_case("laminate", seed=6, nxy=(16, 4), n_ply=3, nparts=(4, 1, 1), nev=8)
    Ke = fem.element_matrices(w)
    A, b, free = fem.assemble(w, Ke)
    its = {}
    for name, coarse in (("as", False), ("zem", "zem"), ("geneo", True)):
        g = geneo.GenEO(w, A, Ke, coarse=coarse)
        if name == "zem":
            assert g.NH == 6 * (w.n_sub - 1)
        u, info = pcg.pcg(A, b[:, 0], g.apply, rtol=1e-5, maxit=2000)
        its[name] = info["iters"]
    assert its["as"] > its["zem"] > its["geneo"], its


def test_zem_dimensions_match_the_example_1b_table():
    """The oracle's ZEM coarse space on the Example 1 plate has the coarse
    dimensions the paper prints for N = 4, 8, 16, 32 (tests/golden fixture)."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "example1b_zem_coarse_dims.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    for N, px, py, dim in [[int(v) for v in r] for r in rows]:
        w = gen.example1b_plate((px, py, 1), nxy=(16, 4))
        assert w.n_sub == N
        d = dd.Decomposition(w)
        got = sum(geneo.zem_basis(w, d, j).shape[1] for j in range(w.n_sub))
        assert got == dim, (N, got, dim)


@pytest.mark.parametrize("kind,kw", [
    ("laminate", dict(nxy=(16, 8), n_ply=3, nparts=(4, 2, 1), nev=8, overlap=1)),
    ("laminate", dict(nxy=(16, 8), n_ply=3, nparts=(4, 2, 1), nev=8, overlap=2)),
    ("diffusion", dict(ne=(16, 16, 8), nparts=(4, 4, 1), overlap=2, threshold=0.15, nev_max=16)),
])
def test_smooth_pou_keeps_geneo_robust(kind, kw):
    """The smooth (Sarkis) partition of unity in GenEO on equal subdomains: the
    paper reports little difference from the standard one (at most one
    iteration).  Checked qualitatively at the 1e-5 reduction of its tables: the
    smooth PoU needs at most one iteration more than the standard one and keeps
    the preconditioned condition number O(10).  With overlap 1 the two PoUs
    coincide (the only shared nodes are equidistant from both boundaries)."""
    from oracle import pcg
    w = gen.small_case(kind, seed=7, **kw)
    Ke = fem.element_matrices(w)
    A, b, free = fem.assemble(w, Ke)
    its, kap, X = {}, {}, {}
    for pou in ("standard", "sarkis"):
        w.pou = pou
        g = geneo.GenEO(w, A, Ke)
        u, info = pcg.pcg(A, b[:, 0], g.apply, rtol=1e-5, maxit=2000)
        its[pou], kap[pou], X[pou] = info["iters"], info["kappa"], g.dec.X
    assert its["sarkis"] <= its["standard"] + 1, its
    assert kap["sarkis"] < 50, kap
    same = all(np.array_equal(a, c) for a, c in zip(X["standard"], X["sarkis"]))
    assert same == (w.overlap == 1)
