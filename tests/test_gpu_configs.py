"""GPU parity on the named configurations.

c1 (16x16x8 laminate, 2x2x1 subdomains, 10 eigenvectors) is compared with the
oracle end to end.  c2 (60x220x85 SPE10-shaped diffusion, the bench workload,
in the bench's launch configuration) is too large for a full oracle run: the
oracle computes sampled rows of A and b one by one, and the GPU solution is
checked through those rows (sampled residuals), plus properties that hold at
any size (symmetry of M^-1, true residual, deterministic replay).
"""
import dataclasses

import numpy as np
import pytest

from oracle import dd, fem, geneo, pcg
from workloads import generate as gen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _gp():
    import paper_1901_05188_amd as gp
    return gp


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


@pytest.fixture(scope="module")
def c1():
    w = gen.config_c1()
    print(f"[gpu] c1 n_free={w.n_free}", flush=True)
    Ke = fem.element_matrices(w)
    A, b, free = fem.assemble(w, Ke)
    g = geneo.GenEO(w, A, Ke, keep_all=True)
    u_ref, info = pcg.pcg(A, b[:, 0], g.apply, rtol=1e-12, maxit=500)
    prob = _gp().Problem.from_workload(w)
    pc = _gp().Preconditioner.from_workload(prob, w)
    return dict(w=w, A=A, b=b, g=g, u_ref=u_ref, info=info, prob=prob, pc=pc)


def test_c1_matvec_and_load(c1):
    A, b, prob = c1["A"], c1["b"], c1["prob"]
    x = np.random.default_rng(0).standard_normal(prob.n_free)
    y = torch.zeros((1, prob.n_free), dtype=torch.float64, device=DEV)
    prob.matvec(_t(x[None, :]), y)
    scale = abs(A) @ np.abs(x)
    assert np.all(np.abs(y[0].cpu().numpy() - A @ x) <= 1e-12 * scale)
    bb = torch.zeros((1, prob.n_free), dtype=torch.float64, device=DEV)
    prob.rhs(bb)
    assert np.allclose(bb[0].cpu().numpy(), b[:, 0], rtol=1e-12, atol=1e-14 * np.abs(b).max())


def test_c1_eigenvalues(c1):
    from tests import oracle_runs as orc
    g, pc, w = c1["g"], c1["pc"], c1["w"]
    orc.check_eigenvalues(w, g, pc.eigenvalues)
    floating = 0
    for j in range(w.n_sub):
        assert g.m[j] == 10
        floating += int(np.sum(np.abs(g.lam[j][:11]) < 1e-9 * abs(g.lam[j][10])) == 6)
    assert floating == 2        # two of the four subdomains do not touch the clamp


def test_c1_solution_iterations_kappa(c1):
    prob, pc, b, u_ref, info = c1["prob"], c1["pc"], c1["b"], c1["u_ref"], c1["info"]
    bt = _t(b[:, 0][None, :])
    x = torch.zeros_like(bt)
    st, rep = _gp().solve(prob, pc, bt, x, rtol=1e-12, maxit=500)
    u = x[0].cpu().numpy()
    print(f"[gpu] c1 iters {rep[0]['iters']} (oracle {info['iters']}) kappa {rep[0]['cond_est']:.2f}")
    assert np.linalg.norm(u - u_ref) <= 1e-8 * np.linalg.norm(u_ref)
    # the un-restarted PCG sequence is the oracle's algorithm
    assert abs(rep[0]["iters_first"] - info["iters"]) <= max(1, int(0.02 * info["iters"]))
    assert abs(rep[0]["cond_est"] - info["kappa"]) <= 1e-3 * info["kappa"]


def test_c1_mixed_precision(c1):
    w, prob, b, u_ref = c1["w"], c1["prob"], c1["b"], c1["u_ref"]
    pc32 = _gp().Preconditioner.from_workload(prob, w, local_prec=32)
    bt = _t(b[:, 0][None, :])
    x = torch.zeros_like(bt)
    st, rep = _gp().solve(prob, pc32, bt, x, rtol=1e-12, maxit=500)
    u = x[0].cpu().numpy()
    assert np.linalg.norm(u - u_ref) <= 1e-7 * np.linalg.norm(u_ref)


@pytest.fixture(scope="module")
def c2():
    w = gen.config_c2()
    print(f"[gpu] c2 n_free={w.n_free}", flush=True)
    prob = _gp().Problem.from_workload(w)
    pc = _gp().Preconditioner.from_workload(prob, w)
    rng = np.random.default_rng(7)
    rows = np.sort(rng.choice(w.n_free, size=60, replace=False))
    sampled = fem.assemble_rows(w, rows)
    return dict(w=w, prob=prob, pc=pc, rows=rows, sampled=sampled)


def test_c2_sampled_rows_of_A_and_b(c2):
    prob, rows, sampled = c2["prob"], c2["rows"], c2["sampled"]
    x = np.random.default_rng(1).standard_normal(prob.n_free)
    y = torch.zeros((1, prob.n_free), dtype=torch.float64, device=DEV)
    prob.matvec(_t(x[None, :]), y)
    bb = torch.zeros((1, prob.n_free), dtype=torch.float64, device=DEV)
    prob.rhs(bb)
    y, bb = y[0].cpu().numpy(), bb[0].cpu().numpy()
    for r, (cols, vals, bv) in zip(rows, sampled):
        assert abs(y[r] - vals @ x[cols]) <= 1e-12 * (np.abs(vals) @ np.abs(x[cols]))
        assert abs(bb[r] - bv) <= 1e-13 * max(abs(bv), 1e-300)


def test_c2_solution_sampled_residual_and_properties(c2):
    prob, pc, rows, sampled = c2["prob"], c2["pc"], c2["rows"], c2["sampled"]
    b = torch.zeros((1, prob.n_free), dtype=torch.float64, device=DEV)
    prob.rhs(b)
    x = torch.zeros_like(b)
    st, rep = _gp().solve(prob, pc, b, x, rtol=1e-8, maxit=3000)
    print(f"[gpu] c2 iters {rep[0]['iters']} kappa {rep[0]['cond_est']:.1f} NH {pc.report['coarse_dim']} "
          f"true_rel_res {rep[0]['true_rel_res']:.2e}")
    print(f"[gpu] c2 res_floor {rep[0]['res_floor']:.2e} restarts {rep[0]['restarts']}")
    # the 1e-8 target holds for the true residual b - A x, not only the recursive one
    assert rep[0]["converged"] == 1 and rep[0]["true_rel_res"] <= 1e-8
    xs = x[0].cpu().numpy()
    bs = b[0].cpu().numpy()
    nb = np.linalg.norm(bs)
    # oracle rows: r_i = b_i - A_i x; small against the row scale |A_i| |x|
    for r, (cols, vals, bv) in zip(rows, sampled):
        res = bv - vals @ xs[cols]
        assert abs(res) <= 1e-6 * (np.abs(vals) @ np.abs(xs[cols])) + 1e-9 * nb / np.sqrt(prob.n_free)
    # M^-1 symmetric: u^T M^-1 v = v^T M^-1 u
    rng = np.random.default_rng(3)
    u, v = _t(rng.standard_normal((1, prob.n_free))), _t(rng.standard_normal((1, prob.n_free)))
    mu, mv = torch.zeros_like(u), torch.zeros_like(v)
    pc.apply(u, mu)
    pc.apply(v, mv)
    a1, a2 = float((v * mu).sum()), float((u * mv).sum())
    assert abs(a1 - a2) <= 1e-10 * max(abs(a1), abs(a2))
    # deterministic replay
    x2 = torch.zeros_like(b)
    _gp().solve(prob, pc, b, x2, rtol=1e-8, maxit=3000)
    assert torch.equal(x, x2)


@pytest.fixture(scope="module")
def c3():
    w = gen.config_c3()
    print(f"[gpu] c3 n_free={w.n_free}", flush=True)
    prob = _gp().Problem.from_workload(w)
    pc64 = _gp().Preconditioner.from_workload(prob, w)
    pc32 = _gp().Preconditioner.from_workload(prob, w, local_prec=32)
    rng = np.random.default_rng(8)
    rows = np.sort(rng.choice(w.n_free, size=40, replace=False))
    sampled = fem.assemble_rows(w, rows)
    return dict(w=w, prob=prob, pc64=pc64, pc32=pc32, rows=rows, sampled=sampled)


def test_c3_sampled_rows_and_eigen_counts(c3):
    prob, rows, sampled, pc = c3["prob"], c3["rows"], c3["sampled"], c3["pc64"]
    x = np.random.default_rng(2).standard_normal(prob.n_free)
    y = torch.zeros((1, prob.n_free), dtype=torch.float64, device=DEV)
    prob.matvec(_t(x[None, :]), y)
    bb = torch.zeros((1, prob.n_free), dtype=torch.float64, device=DEV)
    prob.rhs(bb)
    y, bb = y[0].cpu().numpy(), bb[0].cpu().numpy()
    for r, (cols, vals, bv) in zip(rows, sampled):
        assert abs(y[r] - vals @ x[cols]) <= 1e-12 * (np.abs(vals) @ np.abs(x[cols]))
        assert abs(bb[r] - bv) <= 1e-13 * max(abs(bv), 1e-300)
    # 12 eigenvectors per subdomain (more only through cluster completion)
    assert pc.report["coarse_dim"] >= 12 * c3["w"].n_sub


def test_c3_fp64_and_mixed_solves(c3):
    """Both local precisions inside the FP64 outer loop: the true residual meets
    1e-8 or sits at the FP64 rounding floor eps || |A| |x| || (the cantilever
    load of this plate has a floor near 6e-7), and the two solutions agree."""
    prob = c3["prob"]
    b = torch.zeros((1, prob.n_free), dtype=torch.float64, device=DEV)
    prob.rhs(b)
    xs = {}
    for key in ("pc64", "pc32"):
        x = torch.zeros_like(b)
        st, rep = _gp().solve(prob, c3[key], b, x, rtol=1e-8, maxit=3000, check_every=16)
        r = rep[0]
        print(f"[gpu] c3 {key}: iters {r['iters']} (first {r['iters_first']}, restarts {r['restarts']}) "
              f"kappa {r['cond_est']:.1f} true {r['true_rel_res']:.2e} floor {r['res_floor']:.2e}", flush=True)
        assert r["converged"] == 1
        assert r["true_rel_res"] <= max(1e-8, 4 * r["res_floor"])
        xs[key] = x[0].cpu().numpy()
    d = np.linalg.norm(xs["pc64"] - xs["pc32"]) / np.linalg.norm(xs["pc64"])
    print(f"[gpu] c3 mixed vs FP64 solution: {d:.2e}")
    assert d <= 1e-6


def test_c3_precond_symmetric(c3):
    prob, pc = c3["prob"], c3["pc64"]
    rng = np.random.default_rng(4)
    u, v = _t(rng.standard_normal((1, prob.n_free))), _t(rng.standard_normal((1, prob.n_free)))
    mu, mv = torch.zeros_like(u), torch.zeros_like(v)
    pc.apply(u, mu)
    pc.apply(v, mv)
    a1, a2 = float((v * mu).sum()), float((u * mv).sum())
    assert abs(a1 - a2) <= 1e-10 * max(abs(a1), abs(a2))


def test_c5_largest_single_solve():
    """6,054,912-DOF ramped laminate, 1536 subdomains, FP32 local factors inside
    FP64 PCG, 12 eigenvectors each (N_H = 18,432): sampled rows of A and b
    against the oracle, and the solve reaches 1e-8 or the FP64 rounding floor."""
    w = gen.config_c5()
    print(f"[gpu] c5 n_free={w.n_free}", flush=True)
    prob = _gp().Problem.from_workload(w)
    rows = np.sort(np.random.default_rng(9).choice(w.n_free, size=24, replace=False))
    sampled = fem.assemble_rows(w, rows)
    x = np.random.default_rng(3).standard_normal(prob.n_free)
    y = torch.zeros((1, prob.n_free), dtype=torch.float64, device=DEV)
    prob.matvec(_t(x[None, :]), y)
    b = torch.zeros((1, prob.n_free), dtype=torch.float64, device=DEV)
    prob.rhs(b)
    yh, bh = y[0].cpu().numpy(), b[0].cpu().numpy()
    for r, (cols, vals, bv) in zip(rows, sampled):
        assert abs(yh[r] - vals @ x[cols]) <= 1e-12 * (np.abs(vals) @ np.abs(x[cols]))
        assert abs(bh[r] - bv) <= 1e-13 * max(abs(bv), 1e-300) + 1e-300
    pc = _gp().Preconditioner.from_workload(prob, w, local_prec=32)
    assert pc.report["coarse_dim"] >= 12 * w.n_sub
    xs = torch.zeros_like(b)
    st, rep = _gp().solve(prob, pc, b, xs, rtol=1e-8, maxit=3000, check_every=16)
    r = rep[0]
    print(f"[gpu] c5 iters {r['iters']} kappa {r['cond_est']:.1f} NH {pc.report['coarse_dim']} "
          f"true {r['true_rel_res']:.2e} floor {r['res_floor']:.2e}", flush=True)
    assert r["converged"] == 1
    assert r["true_rel_res"] <= max(1e-8, 4 * r["res_floor"])
    pc.close()
    prob.close()


def test_c4_serving_catalogue_sample():
    """Serving catalogue, one operator of each size (0.2/0.5/1/2 M DOFs), FP32
    local factors inside FP64 PCG, resident together on one request server.
    Twelve requests of the Poisson stream (1-16 patch-traction load cases each)
    are submitted at once: every column reaches 1e-8 (or the FP64 rounding
    floor); sampled rows of a request's load vector against the oracle, and the
    oracle rows' residuals b_i - A_i x of its solution; two requests solved
    again alone give the same bits; one request against FP64 local factors
    (mixed-precision gate 1e-7)."""
    gp = _gp()
    cat = gen.config_c4_catalogue()
    pick = [0, 4, 8, 12]
    ops = []
    for i in pick:
        w = cat[i]
        print(f"[gpu] c4 {w.name} n_free={w.n_free} subdomains={w.n_sub}", flush=True)
        prob = gp.Problem.from_workload(w)
        pc = gp.Preconditioner.from_workload(prob, w, local_prec=32)
        ops.append((w, prob, pc))
    stream = [r for r in gen.c4_requests(16, n_req=200) if r["op"] in pick][:12]
    srv = gp.Server(maxit_cap=3000)
    try:
        ids = [srv.add(p, pc) for (_, p, pc) in ops]
        loads = []
        for r in stream:
            w, p, _ = ops[pick.index(r["op"])]
            b = torch.zeros((r["k"], p.n_free), dtype=torch.float64, device=DEV)
            p.load_vectors(b, traction=gen.patch_tractions(w, r["k"], np.random.default_rng(r["seed"])))
            loads.append((b, torch.zeros_like(b)))
        torch.cuda.synchronize()
        tickets = [srv.submit(ids[pick.index(r["op"])], ops[pick.index(r["op"])][1].n_free, b, x,
                              rtol=1e-8, maxit=3000) for r, (b, x) in zip(stream, loads)]
        reps = []
        for t in tickets:
            st, rep, lat = srv.wait(t)
            assert st == 0
            for c in rep:
                assert c["converged"] == 1
                assert c["true_rel_res"] <= max(1e-8, 4 * c["res_floor"])
            reps.append(rep)
            print(f"[gpu] c4 request: k={len(rep)} latency {lat * 1e3:.0f} ms iters "
                  f"{min(c['iters'] for c in rep)}-{max(c['iters'] for c in rep)}", flush=True)
        for i in (0, len(stream) - 1):
            b, x = loads[i]
            xa = torch.zeros_like(x)
            torch.cuda.synchronize()
            st, rep, lat = srv.wait(srv.submit(ids[pick.index(stream[i]["op"])], b.shape[1], b, xa,
                                               rtol=1e-8, maxit=3000))
            assert torch.equal(xa, x)
    finally:
        srv.close()
    # oracle rows of the smallest operator's first request (first load case)
    i0 = next(i for i, r in enumerate(stream) if r["op"] == pick[0])
    w, p, _ = ops[0]
    trac = gen.patch_tractions(w, stream[i0]["k"], np.random.default_rng(stream[i0]["seed"]))
    w1 = dataclasses.replace(w, traction=trac[: w.ne[0] * w.ne[1] * 3], nrhs=1)
    rows = np.sort(np.random.default_rng(11).choice(w.n_free, size=24, replace=False))
    sampled = fem.assemble_rows(w1, rows)
    b, x = loads[i0]
    bh, xh = b[0].cpu().numpy(), x[0].cpu().numpy()
    nb = np.linalg.norm(bh)
    bound = max(1e-8, 4 * reps[i0][0]["res_floor"]) * nb * 1.01
    for r, (cols, vals, bv) in zip(rows, sampled):
        assert abs(bh[r] - bv) <= 1e-13 * max(abs(bv), np.abs(bh).max())
        assert abs(bv - vals @ xh[cols]) <= bound
    # FP32 against FP64 local factors on the same operator, both run to 1e-11
    pc_f32 = ops[0][2]
    pc64 = gp.Preconditioner.from_workload(p, w, local_prec=64)
    xs = [torch.zeros_like(b[:1]) for _ in range(2)]
    for pcx, xx in zip((pc_f32, pc64), xs):
        st, rep = gp.solve(p, pcx, b[:1], xx, rtol=1e-11, maxit=3000)
        assert rep[0]["converged"] == 1
    err = float(torch.linalg.norm(xs[0] - xs[1]) / torch.linalg.norm(xs[1]))
    served = float(torch.linalg.norm(x[:1] - xs[1]) / torch.linalg.norm(xs[1]))
    print(f"[gpu] c4 FP32-local vs FP64-local solution: {err:.2e}; served (1e-8) vs FP64: {served:.2e}",
          flush=True)
    assert err <= 1e-7
    pc64.close()
    for (_, p, pc) in ops:
        pc.close()
        p.close()
