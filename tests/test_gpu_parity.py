"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Tolerances (FP64 path): assembled A x and b agree to 1e-12 of the row scale
sum_j |A_ij x_j|, and the operators to 32 eps in the normwise measure
||A_gpu x - A x|| / || |A| |x| || (oracle_runs.operator_eta; 2-9 eps observed:
the two sides round their element integrals differently); preconditioner
applications to 1e-10 relative, or three times the case's FP64 condition
where that is larger (tests/oracle_runs.py, minv_gate: on the 3x2x2 laminate
an eps-size perturbation of the element matrices alone moves the oracle's
M^-1 r by about 1e-10), the condition scaled to the measured operator
difference; GenEO eigenvalues to
1e-10 * max(|lambda|, 1e-3 * lambda_cut); solutions to 1e-8 relative after both
sides converge to 1e-12; iteration counts within max(1, 2%).  Mixed precision
(FP32 local factors): solutions to 1e-7.
"""
import dataclasses

import numpy as np
import pytest

from tests import oracle_runs as orc
from oracle import pcg as opcg
from workloads import generate as gen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _gp():
    import paper_1901_05188_amd as gp
    return gp


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    yield


_PROBS = {}


def problem(name):
    if name not in _PROBS:
        w = orc.workload(name)
        print(f"[gpu] assemble {name} ne={w.ne} n_free={w.n_free}", flush=True)
        _PROBS[name] = _gp().Problem.from_workload(w)
    return _PROBS[name]


_ETA = {}


def op_eta(name):
    """operator_eta of the GPU's assembled operator against the oracle's."""
    if name not in _ETA:
        A, b, free, Ke = orc.system(name)
        p = problem(name)
        X = orc.eta_vectors(p.n_free)
        Y = torch.zeros(X.shape, dtype=torch.float64, device=DEV)
        p.matvec(_t(X), Y)
        _ETA[name] = orc.operator_eta(A, X, Y.cpu().numpy())
    return _ETA[name]


_PCS = {}


def precond(name, coarse=True, local_prec=64):
    key = (name, coarse, local_prec)
    if key not in _PCS:
        w = orc.workload(name)
        print(f"[gpu] setup {name} coarse={coarse} prec={local_prec}", flush=True)
        # eigenpairs converged to the rounding level (eig_tol 1e-14; the default
        # 1e-12 is the throughput setting, checked on c1 and the configurations),
        # so that the comparison measures the implementation, not the stopping test
        _PCS[key] = _gp().Preconditioner.from_workload(problem(name), w, local_prec=local_prec,
                                                       coarse=coarse, eig_tol=1e-14)
    return _PCS[key]


ALL = list(orc.CASES)


@pytest.mark.parametrize("name", ALL)
def test_assembled_matvec_matches_oracle(name):
    A, b, free, Ke = orc.system(name)
    p = problem(name)
    assert p.n_free == A.shape[0]
    rng = np.random.default_rng(1)
    X = rng.standard_normal((3, p.n_free))
    Y = torch.zeros((3, p.n_free), dtype=torch.float64, device=DEV)
    p.matvec(_t(X), Y)
    Y = Y.cpu().numpy()
    absA = abs(A)
    for k in range(3):
        ref = A @ X[k]
        scale = absA @ np.abs(X[k])
        assert np.all(np.abs(Y[k] - ref) <= 1e-12 * scale + 1e-300), name
    eta = op_eta(name)
    print(f"[gpu] {name} operator difference {eta / np.finfo(float).eps:.1f} eps", flush=True)
    assert eta <= 32 * np.finfo(float).eps


@pytest.mark.parametrize("name", ALL)
def test_load_vector_matches_oracle(name):
    A, b, free, Ke = orc.system(name)
    p = problem(name)
    out = torch.zeros((p.nrhs, p.n_free), dtype=torch.float64, device=DEV)
    p.rhs(out)
    got = out.cpu().numpy().T
    assert got.shape == b.shape
    assert np.allclose(got, b, rtol=1e-12, atol=1e-14 * np.abs(b).max())


@pytest.mark.parametrize("name", ["lam_ramp_traction", "diff_2x2x2"])
def test_reassembly_gives_the_same_bits(name):
    """gn_reassemble recomputes the element matrices, A and b on the device from
    the inputs the problem keeps (no host arrays): A x and b equal those of the
    first assembly bit for bit, and a preconditioner built afterwards applies
    as one built on a fresh assembly."""
    gp = _gp()
    w = orc.workload(name)
    prob = gp.Problem.from_workload(w)
    try:
        X = _t(np.random.default_rng(2).standard_normal((3, prob.n_free)))
        y0, y1 = torch.zeros_like(X), torch.zeros_like(X)
        b0 = torch.zeros((prob.nrhs, prob.n_free), dtype=torch.float64, device=DEV)
        b1 = torch.zeros_like(b0)
        prob.matvec(X, y0)
        prob.rhs(b0)
        prob.reassemble()
        prob.matvec(X, y1)
        prob.rhs(b1)
        assert torch.equal(y0, y1) and torch.equal(b0, b1)
        pc = gp.Preconditioner.from_workload(prob, w, eig_tol=1e-14)   # the settings of precond()
        try:
            r = X[:1].contiguous()
            z1, z2 = torch.zeros_like(r), torch.zeros_like(r)
            pc.apply(r, z1)
            pc2 = precond(name)
            pc2.apply(r, z2)
            assert torch.equal(z1, z2)
        finally:
            pc.close()
    finally:
        prob.close()


@pytest.mark.parametrize("name", ["lam_2x2", "diff_2x2x2"])
def test_plain_cg_matches_dense_solve(name):
    A, b, free, Ke = orc.system(name)
    p = problem(name)
    u_ref = np.linalg.solve(A.toarray(), b[:, 0])
    bt = _t(b[:, 0][None, :])
    x = torch.zeros_like(bt)
    st, rep = _gp().solve(p, None, bt, x, rtol=1e-12, maxit=20000)
    u = x[0].cpu().numpy()
    assert rep[0]["converged"] == 1
    assert np.linalg.norm(u - u_ref) <= 1e-8 * np.linalg.norm(u_ref)


@pytest.mark.parametrize("name", ALL)
def test_one_level_apply_matches_oracle(name):
    g = orc.geneo_run(name, coarse=False)
    pc = precond(name, coarse=False)
    rng = np.random.default_rng(2)
    r = rng.standard_normal(pc.prob.n_free)
    z = torch.zeros((1, pc.prob.n_free), dtype=torch.float64, device=DEV)
    pc.apply(_t(r[None, :]), z)
    ref = g.apply_as1(r)
    assert np.linalg.norm(z[0].cpu().numpy() - ref) <= 1e-10 * np.linalg.norm(ref)


def _check_eigenvalues(name, pc):
    orc.check_eigenvalues(orc.workload(name), orc.geneo_run(name), pc.eigenvalues)


@pytest.mark.parametrize("name", ALL)
def test_geneo_eigenvalues_and_counts(name):
    _check_eigenvalues(name, precond(name))


@pytest.mark.parametrize("name,block", [("lam_3x2x2_uneven", 16), ("lam_3x2x2_uneven", 40),
                                        ("lam_3x2x2_uneven", 64), ("diff_2x2x2", 40)])
def test_geneo_block_widths(name, block):
    """Eigen blocks of one 16-column block, and wider than one workgroup's 32
    columns (two chunks per subdomain, the last one partial at 40): the block
    solves take their other workgroup shapes and must give the same pairs."""
    w = orc.workload(name)
    print(f"[gpu] setup {name} eig_block={block}", flush=True)
    pc = _gp().Preconditioner.from_workload(problem(name), w, eig_block=block, eig_tol=1e-14)
    try:
        _check_eigenvalues(name, pc)
    finally:
        pc.close()


@pytest.mark.parametrize("name", ALL)
def test_two_level_apply_matches_oracle(name):
    g = orc.geneo_run(name)
    pc = precond(name)
    rng = np.random.default_rng(3)
    r = rng.standard_normal(pc.prob.n_free)
    z = torch.zeros((1, pc.prob.n_free), dtype=torch.float64, device=DEV)
    pc.apply(_t(r[None, :]), z)
    ref = g.apply(r)
    err = np.linalg.norm(z[0].cpu().numpy() - ref) / np.linalg.norm(ref)
    tol = orc.minv_gate(name, seed=3, eta=op_eta(name))
    print(f"[gpu] {name} M^-1 r rel err {err:.2e} (gate {tol:.1e}, FP64 condition "
          f"{orc.minv_eps_sensitivity(name, True, 3):.1e})", flush=True)
    assert err <= tol


@pytest.mark.parametrize("name", ALL)
def test_geneo_pcg_solution_and_iterations(name):
    A, b, free, Ke = orc.system(name)
    u_ref, info = orc.pcg_run(name)
    pc = precond(name)
    p = pc.prob
    bt = _t(b.T)
    x = torch.zeros_like(bt)
    st, rep = _gp().solve(p, pc, bt, x, rtol=1e-12, maxit=2000)
    u = x[0].cpu().numpy()
    assert rep[0]["converged"] == 1
    assert np.linalg.norm(u - u_ref) <= 1e-8 * np.linalg.norm(u_ref)
    # the un-restarted PCG sequence is the oracle's algorithm
    assert abs(rep[0]["iters_first"] - info["iters"]) <= max(1, int(0.02 * info["iters"]))
    assert abs(rep[0]["cond_est"] - info["kappa"]) <= 1e-3 * info["kappa"]


@pytest.mark.parametrize("name", ALL)
def test_zero_energy_mode_coarse_space_matches_oracle(name):
    """Zero-energy-mode coarse space (the paper's ZEM comparison): the same
    coarse dimension and per-subdomain counts as the oracle, M^-1 r to 1e-10
    (the correction does not depend on the basis of the span), the PCG
    solution at 1e-12 (1e-8), and the iteration count and CG-Lanczos kappa at
    the 1e-5 residual reduction of the paper's Example 1b table (max(1, 2 %),
    1e-2).  The count is compared there and not at 1e-12: with ZEM the
    preconditioned kappa is in the thousands, and past 1e-8 the finite-precision
    CG trajectory (loss of orthogonality) shifts by several percent under
    rounding-level changes of M^-1, the oracle against itself included."""
    g = orc.geneo_run(name, coarse="zem")
    pc = precond(name, coarse="zem")
    assert pc.report["coarse_dim"] == g.NH
    for j in range(orc.workload(name).n_sub):
        lam, m = pc.eigenvalues(j)
        assert m == g.m[j] and len(lam) == 0
    rng = np.random.default_rng(5)
    r = rng.standard_normal(pc.prob.n_free)
    z = torch.zeros((1, pc.prob.n_free), dtype=torch.float64, device=DEV)
    pc.apply(_t(r[None, :]), z)
    ref = g.apply(r)
    err = np.linalg.norm(z[0].cpu().numpy() - ref) / np.linalg.norm(ref)
    print(f"[gpu] {name} ZEM N_H {g.NH} M^-1 r rel err {err:.2e}", flush=True)
    assert err <= 1e-10
    A, b, free, Ke = orc.system(name)
    u_ref, info = opcg.pcg(A, b[:, 0], g.apply, rtol=1e-12, maxit=3000)
    bt = _t(b.T[:1])
    x = torch.zeros_like(bt)
    st, rep = _gp().solve(pc.prob, pc, bt, x, rtol=1e-12, maxit=3000)
    assert rep[0]["converged"] == 1
    assert np.linalg.norm(x[0].cpu().numpy() - u_ref) <= 1e-8 * np.linalg.norm(u_ref)
    u5, info5 = opcg.pcg(A, b[:, 0], g.apply, rtol=1e-5, maxit=3000)
    x.zero_()
    st, rep5 = _gp().solve(pc.prob, pc, bt, x, rtol=1e-5, maxit=3000)
    print(f"[gpu] {name} ZEM iterations at 1e-5: {rep5[0]['iters_first']} (oracle {info5['iters']}), "
          f"kappa {rep5[0]['cond_est']:.1f} (oracle {info5['kappa']:.1f}); at 1e-12: "
          f"{rep[0]['iters_first']} (oracle {info['iters']})", flush=True)
    assert abs(rep5[0]["iters_first"] - info5["iters"]) <= max(1, int(0.02 * info5["iters"]))
    assert abs(rep5[0]["cond_est"] - info5["kappa"]) <= 1e-2 * info5["kappa"]


@pytest.mark.parametrize("name", ["lam_3x2x2_uneven", "diff_2x2x2"])
@pytest.mark.parametrize("local_prec", [64, 32])
def test_matrix_core_local_kernel_single_column(name, local_prec):
    """Single-column solves through the 16-column matrix-core kernel (the path
    taken when a band is too wide for the register-pipelined sweep)."""
    A, b, free, Ke = orc.system(name)
    g = orc.geneo_run(name)
    w = orc.workload(name)
    pc = _gp().Preconditioner.from_workload(problem(name), w, local_prec=local_prec, local_kernel=1,
                                            eig_tol=1e-14)
    rng = np.random.default_rng(6)
    r = rng.standard_normal(pc.prob.n_free)
    z = torch.zeros((1, pc.prob.n_free), dtype=torch.float64, device=DEV)
    pc.apply(_t(r[None, :]), z)
    ref = g.apply(r)
    err = np.linalg.norm(z[0].cpu().numpy() - ref) / np.linalg.norm(ref)
    print(f"[gpu] {name} matrix-core local kernel, prec {local_prec}: M^-1 r rel err {err:.2e}")
    # FP32 factors: M^-1 itself changes at the FP32 level; the solve below is the gate
    assert err <= (orc.minv_gate(name, seed=6, eta=op_eta(name)) if local_prec == 64 else 1e-3), err
    u_ref = np.linalg.solve(A.toarray(), b[:, 0])
    bt = _t(b[:, 0][None, :])
    x = torch.zeros_like(bt)
    st, rep = _gp().solve(pc.prob, pc, bt, x, rtol=1e-12, maxit=2000)
    assert rep[0]["converged"] == 1
    tol = 1e-8 if local_prec == 64 else 1e-7
    assert np.linalg.norm(x[0].cpu().numpy() - u_ref) <= tol * np.linalg.norm(u_ref)


@pytest.mark.parametrize("name", ["lam_2x2", "lam_3x2x2_uneven", "diff_2x2x2"])
def test_mixed_precision_local_solves(name):
    A, b, free, Ke = orc.system(name)
    u_ref = np.linalg.solve(A.toarray(), b[:, 0])
    pc = precond(name, local_prec=32)
    bt = _t(b[:, 0][None, :])
    x = torch.zeros_like(bt)
    st, rep = _gp().solve(pc.prob, pc, bt, x, rtol=1e-12, maxit=2000)
    u = x[0].cpu().numpy()
    assert np.linalg.norm(u - u_ref) <= 1e-7 * np.linalg.norm(u_ref)


def test_repeatable_bitwise():
    pc = precond("lam_3x2x2_uneven")
    rng = np.random.default_rng(4)
    r = _t(rng.standard_normal((1, pc.prob.n_free)))
    z1 = torch.zeros_like(r)
    z2 = torch.zeros_like(r)
    pc.apply(r, z1)
    pc.apply(r, z2)
    assert torch.equal(z1, z2)
    b = torch.zeros((pc.prob.nrhs, pc.prob.n_free), dtype=torch.float64, device=DEV)
    pc.prob.rhs(b)
    x1, x2 = torch.zeros_like(b), torch.zeros_like(b)
    _gp().solve(pc.prob, pc, b, x1, rtol=1e-10)
    _gp().solve(pc.prob, pc, b, x2, rtol=1e-10)
    assert torch.equal(x1, x2)


SMOOTH = ["diff_2x2x2|pou=sarkis", "lam_3x2x2_uneven|overlap=2,pou=sarkis"]


@pytest.mark.parametrize("name", SMOOTH)
def test_smooth_partition_of_unity_matches_oracle(name):
    """The smooth (Sarkis) partition of unity (Section 3.2, Section 3.3.1) on
    overlap-2 decompositions, where it differs from the standard one: GenEO
    eigenvalues and counts (its pencil B = X A_O X and basis X p depend on X),
    two-level M^-1 r, and the PCG solution and iteration count."""
    w = orc.workload(name)
    g = orc.geneo_run(name)
    assert w.pou == "sarkis" and w.overlap == 2
    print(f"[gpu] setup {name}", flush=True)
    pc = _gp().Preconditioner.from_workload(problem(name.partition("|")[0]), w, eig_tol=1e-14)
    try:
        orc.check_eigenvalues(w, g, pc.eigenvalues)
        r = np.random.default_rng(3).standard_normal(w.n_free)
        z = torch.zeros((1, w.n_free), dtype=torch.float64, device=DEV)
        pc.apply(_t(r[None, :]), z)
        ref = g.apply(r)
        err = np.linalg.norm(z[0].cpu().numpy() - ref) / np.linalg.norm(ref)
        tol = orc.minv_gate(name, seed=3, eta=op_eta(name.partition("|")[0]))
        print(f"[gpu] {name} M^-1 r rel err {err:.2e} (gate {tol:.1e})", flush=True)
        assert err <= tol
        A, b, free, Ke = orc.system(name)
        u_ref, info = opcg.pcg(A, b[:, 0], g.apply, rtol=1e-12, maxit=2000)
        bt = _t(b[:, 0][None, :])
        x = torch.zeros_like(bt)
        st, rep = _gp().solve(pc.prob, pc, bt, x, rtol=1e-12, maxit=2000)
        assert np.linalg.norm(x[0].cpu().numpy() - u_ref) <= 1e-8 * np.linalg.norm(u_ref)
        assert abs(rep[0]["iters_first"] - info["iters"]) <= max(1, int(0.02 * info["iters"]))
    finally:
        pc.close()


def test_error_paths():
    gp = _gp()
    w = orc.workload("lam_2x2")
    p = problem("lam_2x2")
    with pytest.raises(gp.GenPCGError) as e:
        gp.Preconditioner(p, w.nparts, w.cuts, overlap=0, nev=4)
    assert e.value.code == -1
    bad = [np.array([0, 3, 2, 8]), w.cuts[1], w.cuts[2]]
    with pytest.raises(gp.GenPCGError):
        gp.Preconditioner(p, (3, 2, 1), bad, overlap=1, nev=4)
    b = torch.zeros((1, p.n_free), dtype=torch.float64, device=DEV)
    p.rhs(b)
    x = torch.zeros_like(b)
    st, rep = gp.solve(p, None, b, x, rtol=1e-12, maxit=1)
    assert st == 1 and rep[0]["iters"] == 1 and rep[0]["converged"] == 0
    # a NaN or an infinity in the right-hand side is refused before any iteration
    for bad_value in (float("nan"), float("inf")):
        bad = b.clone()
        bad[0, 5] = bad_value
        with pytest.raises(gp.GenPCGError) as e:
            gp.solve(p, None, bad, x, rtol=1e-8, maxit=10)
        assert e.value.code == -1 and "NaN" in str(e.value)
    # an eigensolver held to one Rayleigh-Ritz step does not converge
    with pytest.raises(gp.GenPCGError) as e:
        gp.Preconditioner.from_workload(p, w, eig_maxit=1)
    assert e.value.code == -4


def test_indefinite_material_is_not_spd():
    """A Poisson ratio above 1/2 makes the isotropic stiffness indefinite: the
    local Cholesky factorisations meet a non-positive pivot (GN_ERR_NOT_SPD)
    and set-up fails without a handle; every kernel still exits normally."""
    gp = _gp()
    w = gen.small_case("laminate", seed=21, nxy=(8, 6), n_ply=2, nparts=(2, 2, 1), nev=6)
    bad = w.mats.copy()
    bad[:] = gen.iso_consts(10000.0, 0.7)
    prob = gp.Problem.from_workload(dataclasses.replace(w, mats=bad))
    try:
        with pytest.raises(gp.GenPCGError) as e:
            gp.Preconditioner.from_workload(prob, w)
        assert e.value.code == -3
    finally:
        prob.close()


def test_pencil_band_too_wide_is_refused():
    """Two subdomains of a 62 x 30 x 30 diffusion box: each Ibar box has a
    31 x 31-node cross-section, a scalar pencil band of 32 tiles, wider than
    the eigen block solves take (30 tiles; the local band, 32 tiles, still fits
    the batched solves).  Set-up fails with GN_ERR_ARG naming the band, raised
    on the host before any block-solve kernel is launched."""
    gp = _gp()
    w = gen.small_case("diffusion", seed=26, ne=(62, 30, 30), nparts=(2, 1, 1), overlap=1, threshold=0.15,
                       nev_max=8)
    prob = gp.Problem.from_workload(w)
    try:
        with pytest.raises(gp.GenPCGError) as e:
            gp.Preconditioner.from_workload(prob, w)
        assert e.value.code == -1 and "wider than the block solves take" in str(e.value), str(e.value)
    finally:
        prob.close()


@pytest.mark.parametrize("name", ["lam_3x2x2_uneven", "diff_3x3x1"])
def test_graph_replayed_chunks_match_eager_launches(name):
    """CG chunks replayed from a captured HIP graph give the bits of the
    kernel-by-kernel solve: several replays with eager work and synchronisation
    in between, a second chunk length (a new capture), and plain CG."""
    A, b, free, Ke = orc.system(name)
    pc = precond(name)
    p = pc.prob
    bt = _t(b.T[:1])
    ref = torch.zeros_like(bt)
    st, rep0 = _gp().solve(p, pc, bt, ref, rtol=1e-10, maxit=2000, graphs=False)
    y = torch.zeros_like(bt)
    for chunk in (8, 8, 5, 8):
        x = torch.zeros_like(bt)
        st, rep = _gp().solve(p, pc, bt, x, rtol=1e-10, maxit=2000, check_every=chunk, graphs=True)
        assert torch.equal(x, ref), chunk
        assert rep[0]["iters"] == rep0[0]["iters"] and rep[0]["restarts"] == rep0[0]["restarts"]
        p.matvec(x, y)                      # eager work between replays
        torch.cuda.synchronize()
    xe, xg = torch.zeros_like(bt), torch.zeros_like(bt)
    _gp().solve(p, None, bt, xe, rtol=1e-10, maxit=20000, graphs=False)
    _gp().solve(p, None, bt, xg, rtol=1e-10, maxit=20000, graphs=True)
    _gp().solve(p, None, bt, xg, rtol=1e-10, maxit=20000, graphs=True)
    assert torch.equal(xe, xg)


def test_edge_cases_single_subdomain_thin_parts_zero_load_empty_coarse():
    """Degenerate cases: one subdomain (M^-1 = A^-1: PCG converges in one step,
    no coarse space), subdomains one element wide (overlap 1), a zero load
    (x = 0 after no iteration), and a threshold no eigenvalue falls below
    (N_H = 0 although a coarse space was asked for)."""
    from oracle import dd, fem, geneo
    gp = _gp()
    # one subdomain
    w = gen.small_case("laminate", seed=41, nxy=(6, 4), n_ply=2, nparts=(1, 1, 1), nev=4)
    A, b, free = fem.assemble(w)
    prob = gp.Problem.from_workload(w)
    pc = gp.Preconditioner.from_workload(prob, w)
    assert pc.report["coarse_dim"] == 0
    bt = _t(b.T[:1])
    x = torch.zeros_like(bt)
    st, rep = gp.solve(prob, pc, bt, x, rtol=1e-12, maxit=100)
    u = np.linalg.solve(A.toarray(), b[:, 0])
    assert rep[0]["iters_first"] <= 2
    assert np.linalg.norm(x[0].cpu().numpy() - u) <= 1e-10 * np.linalg.norm(u)
    # zero load, single column
    z0 = torch.zeros_like(bt)
    xz = torch.ones_like(bt)
    st, rep = gp.solve(prob, pc, z0, xz, rtol=1e-8, maxit=100)
    assert st == 0 and rep[0]["iters"] == 0 and torch.count_nonzero(xz) == 0
    pc.close()
    prob.close()
    # parts one element wide, uneven; and an empty coarse space
    for cuts, thr in (([np.array([0, 1, 2, 6]), np.array([0, 3, 6]), np.array([0, 4])], 0.15),
                      ([np.array([0, 6]), np.array([0, 3, 6]), np.array([0, 4])], 1e-9)):
        rng = np.random.default_rng(7)
        k = np.exp(rng.normal(0.0, 1.0, 6 * 6 * 4))
        w = gen.diffusion_box((6, 6, 4), k, tuple(len(c) - 1 for c in cuts), cuts=cuts, overlap=1,
                              threshold=thr, nev_max=8, dirichlet_faces=("x0",) if thr > 1e-6 else ("x0", "x1"))
        Ke = fem.element_matrices(w)
        A, b, free = fem.assemble(w, Ke)
        g = geneo.GenEO(w, A, Ke)
        prob = gp.Problem.from_workload(w)
        pc = gp.Preconditioner.from_workload(prob, w)
        assert pc.report["coarse_dim"] == g.NH
        if thr < 1e-6:
            assert g.NH == 0
        r = np.random.default_rng(8).standard_normal(prob.n_free)
        zt = torch.zeros((1, prob.n_free), dtype=torch.float64, device=DEV)
        pc.apply(_t(r[None, :]), zt)
        ref = g.apply(r)
        assert np.linalg.norm(zt[0].cpu().numpy() - ref) <= 1e-10 * np.linalg.norm(ref)
        u_ref, info = opcg.pcg(A, b[:, 0], g.apply, rtol=1e-12, maxit=500)
        bt = _t(b.T[:1])
        x = torch.zeros_like(bt)
        st, rep = gp.solve(prob, pc, bt, x, rtol=1e-12, maxit=500)
        assert np.linalg.norm(x[0].cpu().numpy() - u_ref) <= 1e-8 * np.linalg.norm(u_ref)
        assert abs(rep[0]["iters_first"] - info["iters"]) <= max(1, int(0.02 * info["iters"]))
        pc.close()
        prob.close()


@pytest.mark.parametrize("name", ["lam_2x2", "diff_2x2x2"])
def test_flexible_cg_with_exact_preconditioner_reproduces_pcg(name):
    """Flexible CG (Polak-Ribiere beta) with the exact two-level preconditioner
    takes the iterations of the standard recurrence (the two betas agree for a
    fixed symmetric M^-1) and reaches the same solution."""
    A, b, free, Ke = orc.system(name)
    pc = precond(name)
    bt = _t(b[:, 0][None, :])
    x1, x2 = torch.zeros_like(bt), torch.zeros_like(bt)
    st1, r1 = _gp().solve(pc.prob, pc, bt, x1, rtol=1e-12, maxit=2000)
    st2, r2 = _gp().solve(pc.prob, pc, bt, x2, rtol=1e-12, maxit=2000, flexible=True)
    assert st2 == 0 and abs(r1[0]["iters_first"] - r2[0]["iters_first"]) <= 1
    u1, u2 = x1[0].cpu().numpy(), x2[0].cpu().numpy()
    assert np.linalg.norm(u1 - u2) <= 1e-10 * np.linalg.norm(u1)


@pytest.mark.parametrize("name", ["lam_3x2x2_uneven", "diff_2x2x2"])
def test_inexact_coarse_solve_with_flexible_cg_matches_oracle(name):
    """Section 3.3.3, last paragraph: the coarse system solved by block-Jacobi
    CG on the block-sparse A_H, stopped at a loose 1e-1, inside flexible outer
    CG.  The oracle runs the same inner and outer algorithms: the PCG solution
    agrees to 1e-8 after both converge to 1e-12.  Where the inner CG stops by
    its tolerance, one application M^-1 r is compared (1e-8) and the outer
    iteration counts must agree within max(2, 5 %) (the inner stopping step may
    fall differently under rounding).  On the laminate, whose A_H has a
    condition number of about 1e6, the inner CG runs to its iteration cap in
    every application: 200 CG steps on such a matrix amplify rounding
    differences far beyond any fixed gate, so the preconditioner, and with it
    the outer iteration count, is then a property of the rounding; only the
    converged solution is compared."""
    from oracle import geneo as ogeneo
    w = orc.workload(name)
    A, b, free, Ke = orc.system(name)
    g = ogeneo.GenEO(w, A, Ke, coarse_solve="cg", coarse_rtol=1e-1, coarse_maxit=200)
    u_ref, info = opcg.pcg(A, b[:, 0], g.apply, rtol=1e-12, maxit=2000, flexible=True)
    print(f"[gpu] setup {name} inexact coarse solve", flush=True)
    pc = _gp().Preconditioner.from_workload(problem(name), w, eig_tol=1e-14, coarse_solve=1,
                                            coarse_rtol=1e-1, coarse_maxit=200)
    try:
        r = np.random.default_rng(3).standard_normal(w.n_free)
        z = torch.zeros((1, w.n_free), dtype=torch.float64, device=DEV)
        pc.apply(_t(r[None, :]), z)
        ref = g.apply(r)
        err = np.linalg.norm(z[0].cpu().numpy() - ref) / np.linalg.norm(ref)
        bt = _t(b[:, 0][None, :])
        x = torch.zeros_like(bt)
        st, rep = _gp().solve(pc.prob, pc, bt, x, rtol=1e-12, maxit=2000, flexible=True)
        e = np.linalg.norm(x[0].cpu().numpy() - u_ref) / np.linalg.norm(u_ref)
        print(f"[gpu] {name} inexact coarse: M^-1 r rel err {err:.2e}; flexible PCG iters "
              f"{rep[0]['iters_first']} (oracle {info['iters']}), solution rel err {e:.2e}, inner iterations "
              f"max {max(g.coarse_iters)}", flush=True)
        inner_converged = max(g.coarse_iters) < 200
        if inner_converged:
            assert err <= 1e-8
        assert st == 0 and rep[0]["converged"] == 1
        assert e <= 1e-8
        if inner_converged:
            assert abs(rep[0]["iters_first"] - info["iters"]) <= max(2, int(0.05 * info["iters"]))
    finally:
        pc.close()


@pytest.mark.parametrize("name", ["lam_2x2", "diff_2x2x2", "lam_3x2x2_uneven"])
def test_coarse_basis_matches_oracle(name):
    """gn_precond_coarse_basis (Section 3.3.2: Phi_{i(j,k)} = X^(j) p_k^j padded by
    zeros): N_H columns, subdomain j's block zero outside I_j, and spanning the
    oracle's block: the energy-norm residual of each GPU column off span(oracle
    Phi_j) below 1e-9 (1e-13 to 2e-11 observed; a wrong eigenvector would leave
    O(1)).  The GPU's coarse correction R_H^T A_H^-1 R_H r, taken as the
    difference of the two- and one-level applications, must equal the host's
    dense FP64 recomputation from the GPU's own basis and operator
    (A_H = Phi^T (A Phi) with A Phi from gn_matvec) to the case's M^-1 r gate:
    the A_H build and the coarse solve add nothing beyond FP64 rounding."""
    import scipy.linalg as sla
    w = orc.workload(name)
    g = orc.geneo_run(name)
    A, b, free, Ke = orc.system(name)
    pc = precond(name)
    Phi = pc.coarse_basis()
    assert Phi.shape == (w.n_free, g.NH) and pc.report["coarse_dim"] == g.NH
    d = g.dec
    for j in range(w.n_sub):
        a, c = g.offsets[j], g.offsets[j + 1]
        outside = np.ones(w.n_free, dtype=bool)
        outside[d.I[j]] = False
        assert not np.any(Phi[outside, a:c]), j
        if c == a:
            continue          # no eigenvalue below the threshold on this subdomain
        Po, Pg = g.Phi[:, a:c], Phi[:, a:c]
        coef = np.linalg.solve(Po.T @ (A @ Po), Po.T @ (A @ Pg))
        R = Pg - Po @ coef
        res = np.sqrt(np.einsum("ik,ik->k", R, A @ R) / np.einsum("ik,ik->k", Pg, A @ Pg))
        assert res.max() <= 1e-9, (j, res)
    AP = torch.zeros((g.NH, w.n_free), dtype=torch.float64, device=DEV)
    problem(name).matvec(_t(Phi.T), AP)
    AP = AP.cpu().numpy().T
    AH = Phi.T @ AP
    AH = 0.5 * (AH + AH.T)
    r = np.random.default_rng(3).standard_normal(w.n_free)
    host = Phi @ sla.cho_solve(sla.cho_factor(AH, lower=True), Phi.T @ r)
    z2 = torch.zeros((1, w.n_free), dtype=torch.float64, device=DEV)
    z1 = torch.zeros_like(z2)
    pc.apply(_t(r[None, :]), z2)
    precond(name, coarse=False).apply(_t(r[None, :]), z1)
    gpu = (z2 - z1)[0].cpu().numpy()
    err = np.linalg.norm(gpu - host) / np.linalg.norm(host)
    print(f"[gpu] {name} coarse correction vs host recomputation {err:.2e}", flush=True)
    assert err <= orc.minv_gate(name, seed=3)
