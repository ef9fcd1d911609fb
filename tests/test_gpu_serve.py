"""GPU tests of new load cases and of the request server.

* gn_load_vectors: patch-traction and body-force load vectors on an assembled
  operator against the oracle's element loads (Section 2), element by element.
* Server (gn_server_*): several resident operators, requests of 1-6
  right-hand sides, few slots so that columns queue and enter slots as others
  finish.  Every request's solution must be bit-identical whether it was
  solved alone or in the mix of all requests, and identical to gn_solve's
  batched path (a column's arithmetic does not depend on its slot, on the
  check interval or on the other columns).  Columns against the oracle's PCG
  (solution 1e-8, iterations within max(1, 2 %), CG-Lanczos kappa 1e-3).
  Budget refusal and argument errors.
"""
import dataclasses

import numpy as np
import pytest

from tests import oracle_runs as orc
from oracle import fem, pcg as opcg
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


_OPS = {}


def operator(name, local_prec=64, coarse=True):
    key = (name, local_prec, coarse)
    if key not in _OPS:
        w = orc.workload(name)
        print(f"[gpu-serve] setup {name} prec={local_prec} coarse={coarse}", flush=True)
        prob = _gp().Problem.from_workload(w)
        pc = _gp().Preconditioner.from_workload(prob, w, local_prec=local_prec, coarse=coarse)
        _OPS[key] = (w, prob, pc)
    return _OPS[key]


def _loads(name, prob, k, rng):
    """k load cases: patch tractions on laminates, seeded random vectors on diffusion."""
    w = orc.workload(name)
    b = torch.zeros((k, prob.n_free), dtype=torch.float64, device=DEV)
    if w.pde == 1:
        prob.load_vectors(b, traction=gen.patch_tractions(w, k, rng))
    else:
        b.copy_(_t(rng.standard_normal((k, prob.n_free))))
    torch.cuda.synchronize()
    return b


@pytest.mark.parametrize("name", ["lam_3x2x2_uneven", "lam_ramp_traction"])
def test_load_vectors_match_oracle(name):
    w0, prob, _ = operator(name)
    rng = np.random.default_rng(31)
    k = 3
    trac = gen.patch_tractions(w0, k, rng)
    w = dataclasses.replace(w0, traction=trac, nrhs=k, body=None)
    ref = fem.load_full(w)[w.free_index()]              # (n_free, k)
    out = torch.zeros((k, prob.n_free), dtype=torch.float64, device=DEV)
    prob.load_vectors(out, traction=trac)
    got = out.cpu().numpy().T
    scale = np.abs(ref).max()
    assert scale > 0
    assert np.abs(got - ref).max() <= 1e-13 * scale
    # body force only, one column
    wb = dataclasses.replace(w0, traction=None, nrhs=1, body=np.tile([0.0, 0.3, -1.0], w0.n_elem))
    refb = fem.load_full(wb)[w0.free_index()][:, 0]
    outb = torch.zeros((1, prob.n_free), dtype=torch.float64, device=DEV)
    prob.load_vectors(outb, body=wb.body)
    assert np.abs(outb[0].cpu().numpy() - refb).max() <= 1e-13 * np.abs(refb).max()


def _requests(names, probs, n_req, rng, max_k=6):
    reqs = []
    for i in range(n_req):
        o = int(rng.integers(len(names)))
        k = int(rng.integers(1, max_k + 1))
        reqs.append((o, _loads(names[o], probs[o], k, rng)))
    return reqs


def test_server_alone_equals_mix_and_gn_solve():
    names = ["lam_2x2", "diff_2x2x2", "lam_3x2x2_uneven"]
    ops = [operator(nm) for nm in names]
    probs = [o[1] for o in ops]
    rng = np.random.default_rng(32)
    reqs = _requests(names, probs, 10, rng)
    srv = _gp().Server(slots=4, check_every=4, maxit_cap=3000)
    try:
        ids = [srv.add(o[1], o[2]) for o in ops]
        alone = []
        for i, (o, b) in enumerate(reqs):
            x = torch.zeros_like(b)
            torch.cuda.synchronize()
            t = srv.submit(ids[o], probs[o].n_free, b, x, rtol=1e-10, maxit=3000)
            st, rep, lat = srv.wait(t)
            assert st == 0, (i, st)
            alone.append((x, rep))
            print(f"[gpu-serve] alone req {i} op {names[o]} k={b.shape[0]} iters "
                  f"{[r['iters'] for r in rep]} latency {lat * 1e3:.1f} ms", flush=True)
        mix = [torch.zeros_like(b) for (o, b) in reqs]
        torch.cuda.synchronize()
        tickets = []
        for (o, b), x in zip(reqs, mix):
            tickets.append(srv.submit(ids[o], probs[o].n_free, b, x, rtol=1e-10, maxit=3000))
        for i, t in enumerate(tickets):
            st, rep, lat = srv.wait(t)
            assert st == 0
            assert [r["iters"] for r in rep] == [r["iters"] for r in alone[i][1]], i
            assert [r["restarts"] for r in rep] == [r["restarts"] for r in alone[i][1]], i
            assert torch.equal(mix[i], alone[i][0]), i
    finally:
        srv.close()
    # the same columns through gn_solve (batched, 8-iteration checks, up to 16 slots)
    for i, (o, b) in enumerate(reqs):
        if b.shape[0] < 2:
            continue
        x = torch.zeros_like(b)
        st, rep = _gp().solve(probs[o], ops[o][2], b, x, rtol=1e-10, maxit=3000)
        assert torch.equal(x, alone[i][0]), i


def test_server_columns_match_oracle():
    name = "lam_ramp_traction"
    w, prob, pc = operator(name)
    A, _, _, _ = orc.system(name)
    g = orc.geneo_run(name)
    rng = np.random.default_rng(33)
    b = _loads(name, prob, 5, rng)
    srv = _gp().Server(slots=3, check_every=5)
    try:
        op = srv.add(prob, pc)
        x = torch.zeros_like(b)
        torch.cuda.synchronize()
        st, rep, lat = srv.wait(srv.submit(op, prob.n_free, b, x, rtol=1e-12, maxit=2000))
    finally:
        srv.close()
    assert st == 0
    B, X = b.cpu().numpy(), x.cpu().numpy()
    for c in range(B.shape[0]):
        u_ref, info = opcg.pcg(A, B[c], g.apply, rtol=1e-12, maxit=2000)
        print(f"[gpu-serve] col {c}: iters {rep[c]['iters_first']} (oracle {info['iters']}) "
              f"true {rep[c]['true_rel_res']:.2e}", flush=True)
        assert rep[c]["converged"] == 1
        assert np.linalg.norm(X[c] - u_ref) <= 1e-8 * np.linalg.norm(u_ref), c
        assert abs(rep[c]["iters_first"] - info["iters"]) <= max(1, int(0.02 * info["iters"]))
        assert abs(rep[c]["cond_est"] - info["kappa"]) <= 1e-3 * info["kappa"]


def test_server_one_level_and_plain_cg_operators():
    name = "lam_2x2"
    A, _, _, _ = orc.system(name)
    w, prob1, pc1 = operator(name, coarse=False)
    rng = np.random.default_rng(34)
    b = _loads(name, prob1, 4, rng)
    U = np.linalg.solve(A.toarray(), b.cpu().numpy().T).T
    prob2 = _gp().Problem.from_workload(w)           # a second handle, no preconditioner: plain CG
    b2 = _t(rng.standard_normal((3, prob2.n_free)))
    U2 = np.linalg.solve(A.toarray(), b2.cpu().numpy().T).T
    srv = _gp().Server(slots=2, maxit_cap=20000)
    try:
        o1 = srv.add(prob1, pc1)
        o2 = srv.add(prob2, None)
        x1, x2 = torch.zeros_like(b), torch.zeros_like(b2)
        torch.cuda.synchronize()
        t1 = srv.submit(o1, prob1.n_free, b, x1, rtol=1e-12, maxit=2000)
        t2 = srv.submit(o2, prob2.n_free, b2, x2, rtol=1e-12, maxit=20000)
        assert srv.wait(t1)[0] == 0 and srv.wait(t2)[0] == 0
    finally:
        srv.close()
        prob2.close()
    X1, X2 = x1.cpu().numpy(), x2.cpu().numpy()
    for c in range(4):
        assert np.linalg.norm(X1[c] - U[c]) <= 1e-8 * np.linalg.norm(U[c])
    for c in range(3):
        assert np.linalg.norm(X2[c] - U2[c]) <= 1e-8 * np.linalg.norm(U2[c])


def test_server_budget_and_argument_errors():
    gp = _gp()
    w, prob, pc = operator("lam_2x2")
    nbytes = gp.resident_bytes(prob, pc)
    assert nbytes > 0
    srv = gp.Server(hbm_budget=1 << 20)
    try:
        with pytest.raises(gp.GenPCGError) as e:
            srv.add(prob, pc)
        assert e.value.code == -2
    finally:
        srv.close()
    srv = gp.Server(maxit_cap=100)
    try:
        op = srv.add(prob, pc)
        assert srv.last_add_bytes >= nbytes
        b = torch.zeros((1, prob.n_free), dtype=torch.float64, device=DEV)
        x = torch.zeros_like(b)
        torch.cuda.synchronize()
        with pytest.raises(gp.GenPCGError):
            srv.submit(op, prob.n_free, b, x, maxit=101)
        with pytest.raises(gp.GenPCGError):
            srv.submit(op + 1, prob.n_free, b, x)
        # a zero load finishes with x = 0 after no iteration
        t = srv.submit(op, prob.n_free, b, x, maxit=100)
        st, rep, lat = srv.wait(t)
        assert st == 0 and rep[0]["iters"] == 0 and torch.count_nonzero(x) == 0
        srv.remove(op)
        with pytest.raises(gp.GenPCGError):
            srv.submit(op, prob.n_free, b, x)
    finally:
        srv.close()


def test_server_builds_admits_by_footprint_and_evicts():
    """Operators registered by description (gn_server_register): the server
    builds one when a request needs it and its a-priori footprint fits the
    budget, evicting the least recently used idle server-built operator when
    it does not.  With a budget that holds either operator but not both,
    alternating requests evict and rebuild; a rebuilt operator gives the same
    bits, every column matches the oracle's PCG (1e-8), and the measured
    footprint of each built operator lies within 5 % below its estimate
    (fixed eigenvector counts).  A build reserves its estimate plus 1/32 until
    the measured footprint replaces the reservation."""
    gp = _gp()
    names = ["lam_2x2", "lam_3x2x2_uneven"]
    ws = [orc.workload(n) for n in names]
    est = [gp.footprint(w) for w in ws]
    reserve = [e + e // 32 for e in est]
    budget = max(reserve) + max(reserve) // 200
    # either operator builds alone; neither builds beside the other one resident
    assert all(r <= budget for r in reserve)
    assert all(0.95 * est[1 - i] + reserve[i] > budget for i in range(2))
    srv = gp.Server(hbm_budget=budget, slots=4)
    try:
        ids = []
        for w in ws:
            op, e = srv.register(w)
            ids.append(op)
            assert e == gp.footprint(w)
            assert srv.info(op) == {"resident": False, "builds": 0, "evictions": 0, "bytes": e}
        refs, loads = [], []
        for n in names:
            A, b, free, Ke = orc.system(n)
            u, info = orc.pcg_run(n)
            refs.append(u)
            loads.append(_t(b[:, 0][None, :]))
        torch.cuda.synchronize()
        results = []
        for step, i in enumerate([0, 1, 0, 1]):
            x = torch.zeros_like(loads[i])
            print(f"[gpu-serve] request {step} on {names[i]}", flush=True)
            st, rep, lat = srv.wait(srv.submit(ids[i], ws[i].n_free, loads[i], x, rtol=1e-12, maxit=2000))
            assert st == 0 and rep[0]["converged"] == 1
            u = x[0].cpu().numpy()
            assert np.linalg.norm(u - refs[i]) <= 1e-8 * np.linalg.norm(refs[i])
            results.append(x)
            me, other = srv.info(ids[i]), srv.info(ids[1 - i])
            assert me["resident"] and me["builds"] == step // 2 + 1
            assert not other["resident"]
            assert est[i] * 0.95 <= me["bytes"] <= est[i], (names[i], me["bytes"], est[i])
        assert srv.info(ids[0])["evictions"] == 2 and srv.info(ids[1])["evictions"] == 1
        assert torch.equal(results[0], results[2]) and torch.equal(results[1], results[3])
    finally:
        srv.close()


def test_server_refuses_an_operator_larger_than_its_budget():
    gp = _gp()
    w = orc.workload("lam_2x2")
    srv = gp.Server(hbm_budget=int(gp.footprint(w) * 0.5))
    try:
        with pytest.raises(gp.GenPCGError) as e:
            srv.register(w)
        assert e.value.code == -2
    finally:
        srv.close()
