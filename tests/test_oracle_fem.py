"""Pins of the oracle's element integrals, materials and assembly.

Each test checks the oracle against something other than itself: closed forms
derived independently (1-D tensor products), mechanical invariants (rigid
modes, patch test, uniform-strain energy), tensor symmetries of the rotated
orthotropic stiffness, and load resultants.
"""
import math

import numpy as np
import pytest

from oracle import fem
from workloads import generate as gen

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def unit_cube():
    return fem.LOCAL.astype(float).copy()


def test_unit_cube_laplacian_closed_form():
    # 1-D linear element: stiffness K1 and consistent mass M1 (exact with 2-point Gauss);
    # the trilinear Laplacian is K1(x)M1(y)M1(z) + M1(x)K1(y)M1(z) + M1(x)M1(y)K1(z).
    K1 = np.array([[1.0, -1.0], [-1.0, 1.0]])
    M1 = np.array([[1 / 3, 1 / 6], [1 / 6, 1 / 3]])
    # local node a = ax + 2 ay + 4 az -> kron order (z, y, x)
    ref = np.kron(M1, np.kron(M1, K1)) + np.kron(M1, np.kron(K1, M1)) + np.kron(K1, np.kron(M1, M1))
    K = fem.ke_scalar(unit_cube(), 1.0)
    assert np.allclose(K, ref, atol=1e-15)
    assert np.allclose(12 * K[0], [4, 0, 0, -1, 0, -1, -1, -1], atol=1e-13)


def test_uniform_grid_interior_stencil():
    ne = (4, 4, 4)
    w = gen.diffusion_box(ne, np.ones(64), (1, 1, 1), dirichlet_faces=())
    A = fem.assemble_full(w).toarray()
    c = 2 + 5 * (2 + 5 * 2)                      # node (2,2,2)
    row = A[c]
    assert math.isclose(row[c], 8 / 3, rel_tol=1e-13)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                nz = abs(dx) + abs(dy) + abs(dz)
                v = row[c + dx + 5 * (dy + 5 * dz)]
                expect = {0: 8 / 3, 1: 0.0, 2: -1 / 6, 3: -1 / 12}[nz]
                assert abs(v - expect) < 1e-13
    assert abs(row.sum()) < 1e-13


def test_material_C0_is_inverse_compliance_and_symmetric():
    for consts in (gen.PLY_CONSTS, gen.RESIN_CONSTS):
        C = fem.material_C(consts, 0.0)
        S = fem.compliance(consts)
        assert np.allclose(C @ S, np.eye(6), atol=1e-12)
        assert np.allclose(C, C.T, rtol=1e-14, atol=1e-9)
        assert np.all(np.linalg.eigvalsh(C) > 0)


def test_isotropic_resin_lame_form():
    E, nu = 10000.0, 0.35
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    ref = np.zeros((6, 6))
    ref[:3, :3] = lam
    ref[np.arange(3), np.arange(3)] = lam + 2 * mu
    ref[3, 3] = ref[4, 4] = ref[5, 5] = mu
    assert np.allclose(fem.material_C(gen.RESIN_CONSTS, 0.7), ref, rtol=1e-12, atol=1e-8)


def test_C90_swaps_axes_1_and_2():
    C0 = fem.material_C(gen.PLY_CONSTS, 0.0)
    C90 = fem.material_C(gen.PLY_CONSTS, math.pi / 2)
    perm = [1, 0, 2, 4, 3, 5]          # 11<->22, 23<->13
    assert np.allclose(C90, C0[np.ix_(perm, perm)], rtol=1e-12, atol=1e-8)


def test_rotation_preserves_mandel_spectrum():
    D = np.diag([1, 1, 1, math.sqrt(2), math.sqrt(2), math.sqrt(2)])
    ref = np.linalg.eigvalsh(D @ fem.material_C(gen.PLY_CONSTS, 0.0) @ D)
    for th, tl in [(0.3, 0.0), (math.pi / 4, 0.0), (-math.pi / 4, 0.17), (1.1, -0.4)]:
        ev = np.linalg.eigvalsh(D @ fem.material_C(gen.PLY_CONSTS, th, tl) @ D)
        assert np.allclose(ev, ref, rtol=1e-12)


def test_plus_minus_45_are_mirror_images():
    Cp = fem.material_C(gen.PLY_CONSTS, math.pi / 4)
    Cm = fem.material_C(gen.PLY_CONSTS, -math.pi / 4)
    # reflection y -> -y flips the sign of the 23 and 12 shear couplings with 11/22/33/13
    s = np.array([1, 1, 1, -1, 1, -1.0])
    assert np.allclose(Cm, s[:, None] * Cp * s[None, :], rtol=1e-12, atol=1e-8)


def _homog_laminate(ramp=None, theta=0.5, tilt=0.0):
    layers = [("ply", math.degrees(theta), 2, 0.5), ("ply", math.degrees(theta), 1, 0.3)]
    w = gen.laminate_plate((3, 4), (3.0, 2.0), layers, nparts=(1, 1, 1), clamp_x0=False,
                           body=None, ramp=ramp)
    w.elem_mat[:] = 0
    if tilt:
        w.elem_tilt = np.full(w.n_elem, tilt)
    # non-uniform spacing in x and y
    w.xn[0] = np.array([0.0, 0.7, 1.9, 3.0])
    w.xn[1] = np.array([0.0, 0.3, 0.8, 1.6, 2.0])
    return w


@pytest.mark.parametrize("ramp", [None, (0.5, 2.0, math.radians(10.0))])
def test_patch_test_linear_displacement(ramp):
    w = _homog_laminate(ramp=ramp, tilt=0.2 if ramp else 0.0)
    A = fem.assemble_full(w).toarray()
    X = fem.node_xyz(w)
    G = np.array([[0.01, -0.02, 0.005], [0.003, 0.011, -0.007], [-0.004, 0.006, 0.009]])
    u = (X @ G.T + np.array([0.1, -0.2, 0.3])).ravel()
    nn = w.nn
    i, j, k = np.meshgrid(np.arange(nn[0]), np.arange(nn[1]), np.arange(nn[2]), indexing="ij")
    inter_node = np.zeros(nn, bool)
    inter_node[1:-1, 1:-1, 1:-1] = True
    inter_node = np.transpose(inter_node, (2, 1, 0)).ravel()
    I = np.flatnonzero(np.repeat(inter_node, 3))
    Bd = np.flatnonzero(~np.repeat(inter_node, 3))
    uI = np.linalg.solve(A[np.ix_(I, I)], -A[np.ix_(I, Bd)] @ u[Bd])
    assert np.max(np.abs(uI - u[I])) <= 1e-12 * np.max(np.abs(u))


def test_rigid_modes_in_kernel_of_neumann_matrix():
    w = _homog_laminate(ramp=(0.5, 2.0, math.radians(10.0)))
    w.elem_mat[: w.n_elem // 2] = 1           # heterogeneous
    A = fem.assemble_full(w)
    X = fem.node_xyz(w)
    modes = []
    for d in range(3):
        t = np.zeros_like(X)
        t[:, d] = 1
        modes.append(t.ravel())
    for d in range(3):
        om = np.zeros(3)
        om[d] = 1
        modes.append(np.cross(om, X).ravel())
    nA = abs(A).max()
    for m in modes:
        assert np.max(np.abs(A @ m)) <= 1e-11 * nA * np.max(np.abs(m))
    # and nothing else: exactly 6 near-zero eigenvalues
    ev = np.linalg.eigvalsh(A.toarray())
    assert np.sum(ev < 1e-9 * ev[-1]) == 6


def test_uniform_strain_energy():
    w = _homog_laminate(theta=0.9)
    A = fem.assemble_full(w)
    X = fem.node_xyz(w)
    eps = np.array([1e-3, -2e-3, 5e-4, 3e-4, -1e-3, 2e-3])   # engineering Voigt
    E = np.array([[eps[0], eps[5] / 2, eps[4] / 2],
                  [eps[5] / 2, eps[1], eps[3] / 2],
                  [eps[4] / 2, eps[3] / 2, eps[2]]])
    u = (X @ E.T).ravel()
    V = (w.xn[0][-1] - w.xn[0][0]) * (w.xn[1][-1] - w.xn[1][0]) * (w.xn[2][-1] - w.xn[2][0])
    C = fem.material_C(w.mats[0], 0.9)
    assert math.isclose(u @ (A @ u), V * eps @ C @ eps, rel_tol=1e-12)


def test_assembled_system_symmetric_positive_definite():
    w = gen.small_case("laminate", seed=1, nxy=(4, 3), n_ply=2)
    A, b, free = fem.assemble(w)
    Ad = A.toarray()
    assert np.allclose(Ad, Ad.T, rtol=0, atol=1e-10 * abs(Ad).max())
    assert np.linalg.eigvalsh(Ad)[0] > 0


def test_load_resultants():
    w = gen.small_case("laminate", seed=2, nxy=(4, 3), n_ply=2,
                       traction=np.tile([0.0, 0.01, -0.02], 12), body=(0.5, 0.0, -1.0))
    b = fem.load_full(w)[:, 0].reshape(-1, 3)
    V = 4 * 3 * (w.xn[2][-1] - w.xn[2][0])
    area = 4 * 3
    expect = np.array([0.5, 0.0, -1.0]) * V + np.array([0.0, 0.01, -0.02]) * area
    assert np.allclose(b.sum(axis=0), expect, rtol=1e-12, atol=1e-14)


def test_manufactured_solution_second_order():
    errs = []
    for n in (4, 8, 16):
        h = 1.0 / n
        w = gen.diffusion_box((n, n, n), np.ones(n ** 3), (1, 1, 1),
                              dirichlet_faces=("x0", "x1", "y0", "y1", "z0", "z1"), h=h)
        c = (np.arange(n) + 0.5) * h
        cz, cy, cx = np.meshgrid(c, c, c, indexing="ij")
        f = 3 * math.pi ** 2 * np.sin(math.pi * cx) * np.sin(math.pi * cy) * np.sin(math.pi * cz)
        w.body = f.ravel()
        A, b, free = fem.assemble(w)
        u = np.linalg.solve(A.toarray(), b[:, 0])
        X = fem.node_xyz(w)[free]
        ue = np.sin(math.pi * X[:, 0]) * np.sin(math.pi * X[:, 1]) * np.sin(math.pi * X[:, 2])
        errs.append(np.sqrt(np.mean((u - ue) ** 2)))
    rates = [errs[i] / errs[i + 1] for i in range(2)]
    assert all(r > 3.5 for r in rates), (errs, rates)


def test_sampled_rows_equal_full_assembly():
    w = gen.small_case("laminate", seed=3, nxy=(5, 4), n_ply=2,
                       traction=np.tile([0.0, 0.01, -0.02], 20))
    A, b, free = fem.assemble(w)
    rows = [0, 7, 100, w.n_free - 1]
    for r, (cols, vals, bv) in zip(rows, fem.assemble_rows(w, rows)):
        ref = A[r].toarray()[0]
        got = np.zeros_like(ref)
        got[cols] = vals
        assert np.allclose(got, ref, rtol=1e-13, atol=1e-12 * abs(ref).max())
        assert abs(bv - b[r, 0]) <= 1e-13 * max(1.0, abs(b[r, 0]))


@pytest.mark.parametrize("ramp", [(3.0, 7.0, 0.17), (2.5, 6.5, 0.3)])
def test_load_resultant_on_the_ramp(ramp):
    """Top-face traction on the ramped mesh: the resultant of a uniform traction
    g is g times the true area of the tilted top surface.  With the ramp map
    z += tan(angle) (clamp(x, x0, x1) - x0), every Q1 top face is planar (z
    depends on x only, linearly between the face's corner nodes), so its area is
    dx dy sqrt(1 + (dz/dx)^2): dx dy / cos(angle) on the ramp, dx dy on the
    flats, and in between where x0 or x1 falls inside a face (second case)."""
    nx, ny = 10, 4
    g = np.array([0.003, 0.01, -0.02])
    w = gen.small_case("laminate", seed=2, nxy=(nx, ny), n_ply=2, traction=np.tile(g, nx * ny),
                       body=None, ramp=ramp)
    b = fem.load_full(w)[:, 0].reshape(-1, 3)
    x0, x1, ang = ramp
    xn = w.xn[0]
    zt = np.tan(ang) * (np.clip(xn, x0, x1) - x0)          # top-surface lift at each x node
    dx = np.diff(xn)
    dy = np.diff(w.xn[1])
    area = np.sum(np.sqrt(dx ** 2 + np.diff(zt) ** 2)) * np.sum(dy)
    flat = (xn[-1] - xn[0]) * (w.xn[1][-1] - w.xn[1][0])
    assert area > flat * (1 + 1e-3)
    assert np.allclose(b.sum(axis=0), g * area, rtol=1e-12, atol=1e-15)
