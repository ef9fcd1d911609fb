"""The allocation-free load-vector entry point, through the C ABI.

gn_load_vectors_noalloc stages the host loads and the full-numbering load in
the library's static device workspace instead of allocating: its output must
equal gn_load_vectors' bit for bit, on two calls in a row (the second on a
smaller problem with fewer load cases, after the first filled the workspace),
and a request beyond the workspace must be refused with GN_ERR_ARG.
"""
import ctypes as C

import numpy as np
import pytest

from workloads import generate as gen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _lib():
    import paper_1901_05188_amd as gp
    L = gp.lib()
    f = L.gn_load_vectors_noalloc
    f.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.c_int32, C.POINTER(C.c_double), C.c_void_p, C.c_int64,
                  C.c_void_p]
    f.restype = C.c_int32
    return gp, L


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def _both(gp, L, prob, w, nrhs, rng):
    nc = 3 if w.pde == 1 else 1
    trac = rng.normal(0.0, 0.01, nrhs * w.ne[0] * w.ne[1] * nc)
    body = rng.normal(0.0, 1.0, w.n_elem * nc)
    ref = torch.zeros((nrhs, prob.n_free), dtype=torch.float64, device=DEV)
    prob.load_vectors(ref, body=body, traction=trac)
    out = torch.full((nrhs, prob.n_free), np.nan, dtype=torch.float64, device=DEV)
    st = L.gn_load_vectors_noalloc(prob.handle, _ptr(body), nrhs, _ptr(trac), out.data_ptr(), prob.n_free,
                                   torch.cuda.current_stream().cuda_stream)
    assert st == 0, L.gn_last_error()
    torch.cuda.synchronize()
    return ref, out


def test_noalloc_load_vectors_match_the_allocating_entry_point():
    gp, L = _lib()
    torch.cuda.set_device(0)
    rng = np.random.default_rng(17)
    w1 = gen.small_case("laminate", seed=51, nxy=(20, 12), n_ply=4, nparts=(2, 2, 1), nev=6)
    w2 = gen.small_case("laminate", seed=52, nxy=(6, 4), n_ply=2, nparts=(2, 1, 1), nev=4)
    p1 = gp.Problem.from_workload(w1)
    p2 = gp.Problem.from_workload(w2)
    try:
        for prob, w, k in ((p1, w1, 6), (p2, w2, 2)):
            print(f"[gpu] noalloc load vectors: {w.ne} n_free={prob.n_free} nrhs={k}", flush=True)
            ref, out = _both(gp, L, prob, w, k, rng)
            assert torch.equal(ref, out)
        # beyond the static workspace (32 MiB): refused before any device work
        big = 40 * 1024 * 1024 // (8 * (p2.n_free + 1)) + 1
        out = torch.zeros((1, p2.n_free), dtype=torch.float64, device=DEV)
        st = L.gn_load_vectors_noalloc(p2.handle, None, big, None, out.data_ptr(), p2.n_free, None)
        assert st == -1 and b"static workspace" in L.gn_last_error()
    finally:
        p1.close()
        p2.close()
