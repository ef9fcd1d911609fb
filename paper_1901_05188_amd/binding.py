"""ctypes binding of libgenpcg (argument marshalling only).

Every computation happens in the HIP library; this module converts numpy
host arrays and torch device tensors into the plain pointers and sizes of the
C ABI (include/genpcg.h) and turns status codes into exceptions.  Importing it
without the built library raises immediately: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgenpcg.so")

GN_OK, GN_WARN_MAXIT, GN_PENDING = 0, 1, 2
STATUS = {0: "OK", 1: "WARN_MAXIT", 2: "PENDING", -1: "ERR_ARG", -2: "ERR_OOM", -3: "ERR_NOT_SPD",
          -4: "ERR_EIG_NOCONV", -5: "ERR_COARSE_SINGULAR", -6: "ERR_DEVICE", -7: "ERR_BREAKDOWN"}
EXPORTS = ["gn_assemble", "gn_reassemble", "gn_problem_info", "gn_problem_rhs", "gn_load_vectors", "gn_load_vectors_noalloc",
           "gn_matvec",
           "gn_setup_geneo", "gn_precond_eigenvalues", "gn_precond_coarse_basis", "gn_precond_apply", "gn_solve", "gn_footprint", "gn_resident_bytes",
           "gn_server_create", "gn_server_add", "gn_server_register", "gn_server_operator_info",
           "gn_server_remove", "gn_server_submit", "gn_server_wait",
           "gn_server_destroy", "gn_profile_enable", "gn_profile_read", "gn_trim_memory", "gn_destroy_problem",
           "gn_destroy_precond", "gn_last_error"]


class GenPCGError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class gn_grid(C.Structure):
    _fields_ = [("ne", C.c_int32 * 3), ("xn", C.POINTER(C.c_double) * 3),
                ("map_kind", C.c_int32), ("map_par", C.POINTER(C.c_double))]


class gn_material(C.Structure):
    _fields_ = [("pde", C.c_int32), ("n_mat", C.c_int32), ("mat", C.POINTER(C.c_double)),
                ("elem_mat", C.POINTER(C.c_int32)), ("elem_angle", C.POINTER(C.c_double)),
                ("elem_tilt", C.POINTER(C.c_double)), ("elem_k", C.POINTER(C.c_double))]


class gn_loads(C.Structure):
    _fields_ = [("dirichlet", C.POINTER(C.c_uint8)), ("body", C.POINTER(C.c_double)),
                ("nrhs", C.c_int32), ("traction", C.POINTER(C.c_double))]


class gn_dd_opts(C.Structure):
    _fields_ = [("nparts", C.c_int32 * 3), ("cuts", C.POINTER(C.c_int32) * 3),
                ("overlap", C.c_int32), ("nev", C.c_int32), ("threshold", C.c_double),
                ("nev_max", C.c_int32), ("local_prec", C.c_int32), ("coarse", C.c_int32),
                ("shift", C.c_double), ("eig_tol", C.c_double), ("eig_maxit", C.c_int32),
                ("eig_block", C.c_int32), ("eig_filter", C.c_int32), ("local_kernel", C.c_int32),
                ("pou", C.c_int32), ("coarse_solve", C.c_int32), ("coarse_rtol", C.c_double),
                ("coarse_maxit", C.c_int32), ("eig_refine", C.c_int32)]


class gn_setup_report(C.Structure):
    _fields_ = [("n_sub", C.c_int32), ("coarse_dim", C.c_int64), ("eig_iters", C.c_int32),
                ("max_local_n", C.c_int32), ("band_tiles", C.c_int32),
                ("t_local_s", C.c_double), ("t_eigen_s", C.c_double), ("t_coarse_s", C.c_double),
                ("t_total_s", C.c_double), ("hbm_bytes", C.c_int64), ("eig_resid", C.c_double),
                ("eig_solves", C.c_int32), ("t_alloc_s", C.c_double), ("apply_bytes", C.c_double),
                ("apply_tile_bytes", C.c_double), ("local_threads", C.c_int32)]


class gn_solve_opts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("maxit", C.c_int32), ("check_every", C.c_int32),
                ("sequential", C.c_int32), ("graphs", C.c_int32), ("flexible", C.c_int32)]


class gn_server_opts(C.Structure):
    _fields_ = [("hbm_budget", C.c_int64), ("slots", C.c_int32), ("check_every", C.c_int32),
                ("maxit_cap", C.c_int32)]


class gn_solve_report(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("rel_res", C.c_double),
                ("true_rel_res", C.c_double), ("cond_est", C.c_double), ("t_solve_s", C.c_double),
                ("iters_first", C.c_int32), ("restarts", C.c_int32), ("res_floor", C.c_double)]


_lib = None


def lib():
    """Load libgenpcg.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.gn_assemble.argtypes = [C.POINTER(gn_grid), C.POINTER(gn_material), C.POINTER(gn_loads), vp,
                                  C.POINTER(vp)]
        L.gn_reassemble.argtypes = [vp, vp]
        L.gn_problem_info.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                      C.POINTER(C.c_int32)]
        L.gn_problem_rhs.argtypes = [vp, vp, C.c_int64, vp]
        L.gn_load_vectors.argtypes = [vp, C.POINTER(C.c_double), C.c_int32, C.POINTER(C.c_double), vp,
                                      C.c_int64, vp]
        L.gn_matvec.argtypes = [vp, vp, vp, C.c_int32, C.c_int64, vp]
        L.gn_resident_bytes.argtypes = [vp, vp, C.POINTER(C.c_int64)]
        L.gn_footprint.argtypes = [C.POINTER(gn_grid), C.c_int32, C.POINTER(gn_dd_opts), C.POINTER(C.c_int64)]
        L.gn_server_register.argtypes = [vp, C.POINTER(gn_grid), C.POINTER(gn_material), C.POINTER(gn_loads),
                                         C.POINTER(gn_dd_opts), C.POINTER(C.c_int32), C.POINTER(C.c_int64)]
        L.gn_server_operator_info.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                              C.POINTER(C.c_int32), C.POINTER(C.c_int64)]
        L.gn_server_create.argtypes = [C.POINTER(gn_server_opts), C.POINTER(vp)]
        L.gn_server_add.argtypes = [vp, vp, vp, C.POINTER(C.c_int32), C.POINTER(C.c_int64)]
        L.gn_server_remove.argtypes = [vp, C.c_int32]
        L.gn_server_submit.argtypes = [vp, C.c_int32, vp, vp, C.c_int32, C.c_int64, C.c_double, C.c_int32,
                                       C.POINTER(C.c_int64)]
        L.gn_server_wait.argtypes = [vp, C.c_int64, C.c_double, C.POINTER(gn_solve_report),
                                     C.POINTER(C.c_double)]
        L.gn_server_destroy.argtypes = [vp]
        L.gn_server_destroy.restype = None
        L.gn_setup_geneo.argtypes = [vp, C.POINTER(gn_dd_opts), vp, C.POINTER(vp),
                                     C.POINTER(gn_setup_report)]
        L.gn_precond_eigenvalues.argtypes = [vp, C.c_int32, C.POINTER(C.c_double), C.c_int32,
                                             C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.gn_precond_apply.argtypes = [vp, vp, vp, vp]
        L.gn_solve.argtypes = [vp, vp, vp, vp, C.c_int32, C.c_int64, C.POINTER(gn_solve_opts), vp,
                               C.POINTER(gn_solve_report)]
        L.gn_profile_enable.argtypes = [C.c_int32]
        L.gn_trim_memory.argtypes = [C.POINTER(C.c_int64)]
        L.gn_profile_read.argtypes = [C.c_char_p, C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                      C.POINTER(C.c_double)]
        L.gn_destroy_problem.argtypes = [vp]
        L.gn_destroy_problem.restype = None
        L.gn_destroy_precond.argtypes = [vp]
        L.gn_destroy_precond.restype = None
        L.gn_last_error.restype = C.c_char_p
        for f in EXPORTS:
            if f not in ("gn_destroy_problem", "gn_destroy_precond", "gn_server_destroy", "gn_last_error"):
                getattr(L, f).restype = C.c_int32
        _lib = L
    return _lib


def _check(code: int) -> int:
    if code < 0:
        raise GenPCGError(code, lib().gn_last_error().decode())
    return code


def _dptr(a: Optional[np.ndarray], ctype):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(ctype))


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _tensor_ptr(t) -> int:
    return int(t.data_ptr())


def _spec_structs(ne, xn, pde, *, mats=None, elem_mat=None, elem_angle=None, elem_tilt=None, elem_k=None,
                  dirichlet, body=None, nrhs=1, traction=None, map_kind=0, map_par=None):
    """gn_grid, gn_material and gn_loads for host arrays; returns them with the
    arrays they point into (kept alive by the caller for the call)."""
    keep = []

    def arr(a, dt):
        if a is None:
            return None
        a = np.ascontiguousarray(a, dtype=dt)
        keep.append(a)
        return a

    g = gn_grid()
    for a in range(3):
        g.ne[a] = int(ne[a])
        g.xn[a] = _dptr(arr(xn[a], np.float64), C.c_double)
    g.map_kind = int(map_kind)
    g.map_par = _dptr(arr(map_par, np.float64), C.c_double)
    m = gn_material()
    m.pde = int(pde)
    mats_a = arr(mats, np.float64)
    m.n_mat = 0 if mats_a is None else mats_a.shape[0]
    m.mat = _dptr(mats_a, C.c_double)
    m.elem_mat = _dptr(arr(elem_mat, np.int32), C.c_int32)
    m.elem_angle = _dptr(arr(elem_angle, np.float64), C.c_double)
    m.elem_tilt = _dptr(arr(elem_tilt, np.float64), C.c_double)
    m.elem_k = _dptr(arr(elem_k, np.float64), C.c_double)
    l = gn_loads()
    l.dirichlet = _dptr(arr(dirichlet, np.uint8), C.c_uint8)
    l.body = _dptr(arr(body, np.float64), C.c_double)
    l.nrhs = int(nrhs)
    l.traction = _dptr(arr(traction, np.float64), C.c_double)
    return g, m, l, keep


def _workload_spec(w):
    return dict(ne=w.ne, xn=w.xn, pde=w.pde, mats=w.mats, elem_mat=w.elem_mat, elem_angle=w.elem_angle,
                elem_tilt=w.elem_tilt, elem_k=w.elem_k, dirichlet=w.dirichlet, body=w.body, nrhs=w.nrhs,
                traction=w.traction, map_kind=w.map_kind, map_par=w.map_par)


def _dd_struct(nparts, cuts, overlap=1, nev=0, threshold=0.0, nev_max=0, local_prec=64, coarse=True, shift=0.0,
               eig_tol=0.0, eig_maxit=0, eig_block=0, eig_filter=0, local_kernel=0, pou=0, coarse_solve=0,
               coarse_rtol=0.0, coarse_maxit=0, eig_refine=0):
    o = gn_dd_opts()
    keep = []
    for a in range(3):
        o.nparts[a] = int(nparts[a])
        c = np.ascontiguousarray(cuts[a], dtype=np.int32)
        keep.append(c)
        o.cuts[a] = _dptr(c, C.c_int32)
    o.overlap, o.nev, o.threshold, o.nev_max = int(overlap), int(nev), float(threshold), int(nev_max)
    o.local_prec = int(local_prec)
    o.coarse = {"geneo": 1, "zem": 2, "none": 0}[coarse] if isinstance(coarse, str) else int(coarse)
    o.shift, o.eig_tol, o.eig_maxit = float(shift), float(eig_tol), int(eig_maxit)
    o.eig_block, o.eig_filter = int(eig_block), int(eig_filter)
    o.local_kernel = int(local_kernel)
    o.pou = {"standard": 0, "sarkis": 1}[pou] if isinstance(pou, str) else int(pou)
    o.coarse_solve = {"exact": 0, "cg": 1}[coarse_solve] if isinstance(coarse_solve, str) else int(coarse_solve)
    o.coarse_rtol, o.coarse_maxit = float(coarse_rtol), int(coarse_maxit)
    o.eig_refine = int(eig_refine)
    return o, keep


def _workload_dd(w, **kw):
    kw.setdefault("pou", getattr(w, "pou", "standard"))
    return _dd_struct(w.nparts, w.cuts, overlap=w.overlap, nev=w.nev, threshold=w.threshold, nev_max=w.nev_max,
                      **kw)


class Problem:
    """Assembled system on the device (gn_assemble)."""

    def __init__(self, ne, xn, pde, *, mats=None, elem_mat=None, elem_angle=None, elem_tilt=None,
                 elem_k=None, dirichlet, body=None, nrhs=1, traction=None, map_kind=0,
                 map_par=None, stream=None):
        g, m, l, keep = _spec_structs(ne, xn, pde, mats=mats, elem_mat=elem_mat, elem_angle=elem_angle,
                                      elem_tilt=elem_tilt, elem_k=elem_k, dirichlet=dirichlet, body=body,
                                      nrhs=nrhs, traction=traction, map_kind=map_kind, map_par=map_par)
        h = C.c_void_p()
        _check(lib().gn_assemble(C.byref(g), C.byref(m), C.byref(l), _stream(stream), C.byref(h)))
        self.handle = h
        nf, nnz, nr = C.c_int64(), C.c_int64(), C.c_int32()
        _check(lib().gn_problem_info(h, C.byref(nf), C.byref(nnz), C.byref(nr)))
        self.n_free, self.nnz, self.nrhs = nf.value, nnz.value, nr.value

    @classmethod
    def from_workload(cls, w, stream=None) -> "Problem":
        return cls(w.ne, w.xn, w.pde, mats=w.mats, elem_mat=w.elem_mat, elem_angle=w.elem_angle,
                   elem_tilt=w.elem_tilt, elem_k=w.elem_k, dirichlet=w.dirichlet, body=w.body,
                   nrhs=w.nrhs, traction=w.traction, map_kind=w.map_kind, map_par=w.map_par,
                   stream=stream)

    def reassemble(self, stream=None):
        """Recompute the element matrices, A and b on the device from the inputs
        the problem holds (gn_reassemble: no host transfer)."""
        _check(lib().gn_reassemble(self.handle, _stream(stream)))
        return self

    def rhs(self, out, stream=None):
        """Copy the assembled load into a (nrhs, n_free) float64 CUDA tensor (column = row of out)."""
        assert out.is_cuda and out.dtype.is_floating_point and out.is_contiguous()
        assert out.shape[-1] == self.n_free and out.numel() >= self.nrhs * self.n_free
        _check(lib().gn_problem_rhs(self.handle, _tensor_ptr(out), self.n_free, _stream(stream)))
        return out

    def load_vectors(self, out, body=None, traction=None, stream=None):
        """Load vectors of new load cases into a (nrhs, n_free) float64 CUDA tensor.

        body: (n_elem * ncomp,) host array added to every column, or None;
        traction: (nrhs * ne[0] * ne[1] * ncomp,) host array, layout [rhs][face][comp], or None."""
        nrhs = 1 if out.dim() == 1 else out.shape[0]
        assert out.is_cuda and out.dtype.is_floating_point and out.is_contiguous()
        assert out.shape[-1] == self.n_free
        bd = None if body is None else np.ascontiguousarray(body, dtype=np.float64)
        tr = None if traction is None else np.ascontiguousarray(traction, dtype=np.float64)
        _check(lib().gn_load_vectors(self.handle, _dptr(bd, C.c_double), nrhs, _dptr(tr, C.c_double),
                                     _tensor_ptr(out), self.n_free, _stream(stream)))
        return out

    def load_vectors_noalloc(self, out, body=None, traction=None, stream=None):
        """load_vectors through gn_load_vectors_noalloc: the library's static
        device workspace instead of temporary allocations (32 MiB per device;
        concurrent calls on one device race)."""
        nrhs = 1 if out.dim() == 1 else out.shape[0]
        assert out.is_cuda and out.dtype.is_floating_point and out.is_contiguous()
        assert out.shape[-1] == self.n_free
        bd = None if body is None else np.ascontiguousarray(body, dtype=np.float64)
        tr = None if traction is None else np.ascontiguousarray(traction, dtype=np.float64)
        _check(lib().gn_load_vectors_noalloc(self.handle, _dptr(bd, C.c_double), nrhs, _dptr(tr, C.c_double),
                                             _tensor_ptr(out), self.n_free, _stream(stream)))
        return out

    def matvec(self, x, y, stream=None):
        """y = A x for (ncol, n_free) float64 CUDA tensors."""
        ncol = 1 if x.dim() == 1 else x.shape[0]
        assert x.shape == y.shape and x.shape[-1] == self.n_free and x.is_contiguous() and y.is_contiguous()
        _check(lib().gn_matvec(self.handle, _tensor_ptr(x), _tensor_ptr(y), ncol, self.n_free,
                               _stream(stream)))
        return y

    def close(self):
        if getattr(self, "handle", None):
            lib().gn_destroy_problem(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Preconditioner:
    """GenEO two-level additive Schwarz preconditioner (gn_setup_geneo).

    coarse: True / 1 / "geneo" (GenEO), "zem" / 2 (zero-energy modes), False / 0 / "none" (one level)."""

    def __init__(self, prob: Problem, nparts: Sequence[int], cuts, overlap=1, nev=0, threshold=0.0,
                 nev_max=0, local_prec=64, coarse=True, shift=0.0, eig_tol=0.0, eig_maxit=0,
                 eig_block=0, eig_filter=0, local_kernel=0, pou=0, coarse_solve=0, coarse_rtol=0.0,
                 coarse_maxit=0, eig_refine=0, stream=None):
        o, keep = _dd_struct(nparts, cuts, overlap, nev, threshold, nev_max, local_prec, coarse, shift, eig_tol,
                             eig_maxit, eig_block, eig_filter, local_kernel, pou, coarse_solve, coarse_rtol,
                             coarse_maxit, eig_refine)
        rep = gn_setup_report()
        h = C.c_void_p()
        _check(lib().gn_setup_geneo(prob.handle, C.byref(o), _stream(stream), C.byref(h), C.byref(rep)))
        self.handle = h
        self.prob = prob
        self.report = {f: getattr(rep, f) for f, _ in gn_setup_report._fields_}

    @classmethod
    def from_workload(cls, prob: Problem, w, local_prec=64, coarse=True, stream=None, **kw):
        kw.setdefault("pou", getattr(w, "pou", "standard"))
        return cls(prob, w.nparts, w.cuts, overlap=w.overlap, nev=w.nev, threshold=w.threshold,
                   nev_max=w.nev_max, local_prec=local_prec, coarse=coarse, stream=stream, **kw)

    def eigenvalues(self, sub: int):
        buf = (C.c_double * 128)()
        m, n = C.c_int32(), C.c_int32()
        _check(lib().gn_precond_eigenvalues(self.handle, int(sub), buf, 128, C.byref(m), C.byref(n)))
        return np.array(buf[: n.value]), m.value

    def coarse_basis(self) -> np.ndarray:
        """The coarse basis Phi as a host array (n_free, N_H) (gn_precond_coarse_basis)."""
        nh = C.c_int64()
        _check(lib().gn_precond_coarse_basis(self.handle, None, 0, C.byref(nh)))
        n_free = self.prob.n_free
        out = np.zeros((nh.value, n_free), dtype=np.float64)   # column-major n_free x N_H
        if nh.value:
            _check(lib().gn_precond_coarse_basis(self.handle, _dptr(out, C.c_double), n_free, None))
        return out.T

    def apply(self, r, z, stream=None):
        assert r.shape == z.shape and r.shape[-1] == self.prob.n_free
        _check(lib().gn_precond_apply(self.handle, _tensor_ptr(r), _tensor_ptr(z), _stream(stream)))
        return z

    def close(self):
        if getattr(self, "handle", None):
            lib().gn_destroy_precond(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve(prob: Problem, pc: Optional[Preconditioner], b, x, rtol=1e-8, maxit=1000, check_every=8,
          stream=None, sequential=False, graphs=True, flexible=False):
    """PCG (x0 = 0) on (nrhs, n_free) float64 CUDA tensors; returns (status, reports).

    Several right-hand sides are solved in batches of up to 16 columns that
    share every launch, unless sequential=True.  graphs=True replays each chunk
    of check_every iterations of a single-column solve from a captured HIP graph."""
    nrhs = 1 if b.dim() == 1 else b.shape[0]
    assert b.shape == x.shape and b.shape[-1] == prob.n_free and b.is_contiguous() and x.is_contiguous()
    o = gn_solve_opts(float(rtol), int(maxit), int(check_every), int(bool(sequential)), int(bool(graphs)),
                      int(bool(flexible)))
    reps = (gn_solve_report * nrhs)()
    st = _check(lib().gn_solve(prob.handle, pc.handle if pc is not None else None, _tensor_ptr(b),
                               _tensor_ptr(x), nrhs, prob.n_free, C.byref(o), _stream(stream), reps))
    return st, [{f: getattr(r, f) for f, _ in gn_solve_report._fields_} for r in reps]


def resident_bytes(prob: Problem, pc: Optional[Preconditioner] = None) -> int:
    """Device bytes held by a problem and (optionally) its preconditioner."""
    b = C.c_int64()
    _check(lib().gn_resident_bytes(prob.handle, pc.handle if pc is not None else None, C.byref(b)))
    return b.value


def footprint(w, local_prec=64, coarse=True, with_precond=True, **kw) -> int:
    """A-priori resident bytes of a workload's operator (and preconditioner)
    as a request server holds them (gn_footprint: host arithmetic only)."""
    g, m, l, keep = _spec_structs(**_workload_spec(w))
    b = C.c_int64()
    if with_precond:
        o, keep2 = _workload_dd(w, local_prec=local_prec, coarse=coarse, **kw)
        _check(lib().gn_footprint(C.byref(g), int(w.pde), C.byref(o), C.byref(b)))
    else:
        _check(lib().gn_footprint(C.byref(g), int(w.pde), None, C.byref(b)))
    return b.value


class Server:
    """Request server (gn_server_*): resident operators, up to `slots` columns
    per operator in every launch, finished columns replaced at each check."""

    def __init__(self, hbm_budget=0, slots=0, check_every=0, maxit_cap=0):
        o = gn_server_opts(int(hbm_budget), int(slots), int(check_every), int(maxit_cap))
        h = C.c_void_p()
        _check(lib().gn_server_create(C.byref(o), C.byref(h)))
        self.handle = h
        self._keep = {}

    def add(self, prob: Problem, pc: Optional[Preconditioner] = None) -> int:
        """Register an operator; returns its id (raises GenPCGError ERR_OOM beyond the budget)."""
        op, by = C.c_int32(), C.c_int64()
        _check(lib().gn_server_add(self.handle, prob.handle, pc.handle if pc is not None else None,
                                   C.byref(op), C.byref(by)))
        self.last_add_bytes = by.value
        return op.value

    def register(self, w, local_prec=64, coarse=True, **kw):
        """Register a workload by its description; the server builds it when a
        request needs it and the budget allows (gn_server_register).  Returns
        (operator id, footprint estimate)."""
        g, m, l, keep = _spec_structs(**_workload_spec(w))
        o, keep2 = _workload_dd(w, local_prec=local_prec, coarse=coarse, **kw)
        op, est = C.c_int32(), C.c_int64()
        _check(lib().gn_server_register(self.handle, C.byref(g), C.byref(m), C.byref(l), C.byref(o),
                                        C.byref(op), C.byref(est)))
        return op.value, est.value

    def info(self, op: int):
        """(resident, builds, evictions, bytes) of an operator."""
        r, b, e, by = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int64()
        _check(lib().gn_server_operator_info(self.handle, int(op), C.byref(r), C.byref(b), C.byref(e),
                                             C.byref(by)))
        return {"resident": bool(r.value), "builds": b.value, "evictions": e.value, "bytes": by.value}

    def remove(self, op: int):
        _check(lib().gn_server_remove(self.handle, int(op)))

    def submit(self, op: int, n_free: int, b, x, rtol=1e-8, maxit=1000) -> int:
        """Queue the rows of (nrhs, n_free) float64 CUDA tensors b -> x; returns a ticket.
        b must be complete on the device (synchronise its producer first)."""
        nrhs = 1 if b.dim() == 1 else b.shape[0]
        assert b.shape == x.shape and b.shape[-1] == n_free and b.is_contiguous() and x.is_contiguous()
        t = C.c_int64()
        _check(lib().gn_server_submit(self.handle, int(op), _tensor_ptr(b), _tensor_ptr(x), nrhs, n_free,
                                      float(rtol), int(maxit), C.byref(t)))
        self._keep[t.value] = (b, x, nrhs)
        return t.value

    def wait(self, ticket: int, timeout=-1.0):
        """Block until the request finishes (or timeout seconds pass: returns None).
        Returns (status, reports, latency_s)."""
        b, x, nrhs = self._keep[ticket]
        reps = (gn_solve_report * nrhs)()
        lat = C.c_double()
        st = lib().gn_server_wait(self.handle, int(ticket), float(timeout), reps, C.byref(lat))
        if st == GN_PENDING:
            return None
        del self._keep[ticket]
        _check(st)
        return st, [{f: getattr(r, f) for f, _ in gn_solve_report._fields_} for r in reps], lat.value

    def close(self):
        if getattr(self, "handle", None):
            lib().gn_server_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def trim_memory() -> int:
    """Return the library's cached idle device blocks to the runtime; bytes released."""
    n = C.c_int64()
    _check(lib().gn_trim_memory(C.byref(n)))
    return n.value


def profile_enable(on: bool = True):
    _check(lib().gn_profile_enable(1 if on else 0))


def profile_read(group: str):
    ms, n, by = C.c_double(), C.c_int64(), C.c_double()
    _check(lib().gn_profile_read(group.encode(), C.byref(ms), C.byref(n), C.byref(by)))
    return ms.value, n.value, by.value
