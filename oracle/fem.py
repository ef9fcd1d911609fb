"""Oracle: Q1 finite elements, material tensors and assembly (FP64, CPU).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows Section 2 of the paper: strain as the symmetric displacement gradient
(eq-strain), generalised Hooke's law with a rotated orthotropic tensor
(eq-hooke and the paragraph after it), the weak form a(u, v) = b(v) (eq-fe) and
its element-wise Gaussian-integrated assembly into A u = b
(eqn:fe_matrix_system); Section 6 gives the scalar Darcy form (eq-fe-darcy).

Readings taken where the paper is silent:
* element: trilinear Q1 hexahedron, 2x2x2 Gauss-Legendre points (+-1/sqrt(3),
  unit weights); traction faces use 2x2 points;
* Voigt order (11, 22, 33, 23, 13, 12) with engineering shear strains;
* the load functional is b(v) = int f.v + int g.v (the sign printed in eq-fe
  conflicts with the strong form eq:strongForm; the strong form is followed);
* Dirichlet DOFs are homogeneous and eliminated (rows and columns dropped).

Pins (tests/test_oracle_fem.py): closed-form unit-cube Laplacian, interior
stencil of the uniform Laplacian, patch test, rigid-body kernel of the Neumann
matrix, uniform-strain energy, C(0) = S^-1, C(90) = C(0) with axes 1 and 2
swapped, rotation invariance of the Mandel-form spectrum, symmetry and
positive definiteness.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

GP = np.array([-1.0, 1.0]) / math.sqrt(3.0)
# local node a <-> (ax, ay, az), a = ax + 2 ay + 4 az
LOCAL = np.array([[a & 1, (a >> 1) & 1, (a >> 2) & 1] for a in range(8)])
XI = 2.0 * LOCAL - 1.0
VOIGT = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]


def shape(xi: np.ndarray):
    """Q1 shape functions N_a(xi) and derivatives dN_a/dxi_d at one point."""
    f = 0.5 * (1.0 + XI * xi[None, :])            # (8,3) 1-D factors
    N = f[:, 0] * f[:, 1] * f[:, 2]
    dN = np.empty((8, 3))
    dN[:, 0] = 0.5 * XI[:, 0] * f[:, 1] * f[:, 2]
    dN[:, 1] = 0.5 * XI[:, 1] * f[:, 0] * f[:, 2]
    dN[:, 2] = 0.5 * XI[:, 2] * f[:, 0] * f[:, 1]
    return N, dN


def quad_points():
    for gz in GP:
        for gy in GP:
            for gx in GP:
                yield np.array([gx, gy, gz]), 1.0


# ---------------------------------------------------------------------------
# geometry
# ---------------------------------------------------------------------------

def ramp_offset(x, map_par):
    """z offset r(x) of the ramp map: continuous, slope tan(angle) on [x0, x1]."""
    x0, x1, ang = map_par
    return np.tan(ang) * (np.clip(x, x0, x1) - x0)


def node_xyz(w) -> np.ndarray:
    """Physical coordinates of all nodes (n_node, 3), x fastest."""
    nx, ny, nz = w.nn
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    X = np.stack([w.xn[0][i.ravel()], w.xn[1][j.ravel()], w.xn[2][k.ravel()]], axis=1)
    if w.map_kind == 1:
        X[:, 2] += ramp_offset(X[:, 0], w.map_par)
    return X


def elem_nodes(w, e: np.ndarray) -> np.ndarray:
    """Global node ids (len(e), 8) of elements e in local order a."""
    nx, ny, _ = w.ne
    ex = e % nx
    ey = (e // nx) % ny
    ez = e // (nx * ny)
    NX, NY = nx + 1, ny + 1
    out = np.empty((len(e), 8), dtype=np.int64)
    for a in range(8):
        ax, ay, az = LOCAL[a]
        out[:, a] = (ex + ax) + NX * ((ey + ay) + NY * (ez + az))
    return out


# ---------------------------------------------------------------------------
# material (eq-hooke; ply rotation by standard tensor rotation)
# ---------------------------------------------------------------------------

def compliance(c) -> np.ndarray:
    """Orthotropic compliance in Voigt form from (E1,E2,E3,G12,G13,G23,nu12,nu13,nu23)."""
    E1, E2, E3, G12, G13, G23, n12, n13, n23 = c
    S = np.zeros((6, 6))
    S[0, 0], S[1, 1], S[2, 2] = 1 / E1, 1 / E2, 1 / E3
    S[0, 1] = S[1, 0] = -n12 / E1
    S[0, 2] = S[2, 0] = -n13 / E1
    S[1, 2] = S[2, 1] = -n23 / E2
    S[3, 3], S[4, 4], S[5, 5] = 1 / G23, 1 / G13, 1 / G12
    return S


def voigt_to_tensor(Cv: np.ndarray) -> np.ndarray:
    C = np.zeros((3, 3, 3, 3))
    for I, (i, j) in enumerate(VOIGT):
        for J, (k, l) in enumerate(VOIGT):
            for (a, b) in {(i, j), (j, i)}:
                for (c, d) in {(k, l), (l, k)}:
                    C[a, b, c, d] = Cv[I, J]
    return C


def tensor_to_voigt(C: np.ndarray) -> np.ndarray:
    Cv = np.zeros((6, 6))
    for I, (i, j) in enumerate(VOIGT):
        for J, (k, l) in enumerate(VOIGT):
            Cv[I, J] = C[i, j, k, l]
    return Cv


def rotation(theta: float, tilt: float = 0.0) -> np.ndarray:
    """Q mapping material axes to global axes: in-plane angle theta about z,
    then a tilt about y taking the x axis to (cos t, 0, sin t)."""
    c, s = math.cos(theta), math.sin(theta)
    Rz = np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])
    ct, st = math.cos(tilt), math.sin(tilt)
    Ry = np.array([[ct, 0.0, -st], [0.0, 1.0, 0.0], [st, 0.0, ct]])
    return Ry @ Rz


def material_C(consts, theta: float = 0.0, tilt: float = 0.0) -> np.ndarray:
    """Rotated stiffness C'_ijkl = Q_ip Q_jq Q_kr Q_ls C_pqrs, in Voigt form."""
    C0 = np.linalg.inv(compliance(consts))
    C0 = 0.5 * (C0 + C0.T)
    Q = rotation(theta, tilt)
    Ct = np.einsum("ip,jq,kr,ls,pqrs->ijkl", Q, Q, Q, Q, voigt_to_tensor(C0))
    return tensor_to_voigt(Ct)


# ---------------------------------------------------------------------------
# element integrals (eq-fe, eq-fe-darcy; Gaussian integration)
# ---------------------------------------------------------------------------

def _grad_det(Xe: np.ndarray, xi: np.ndarray):
    """Physical shape gradients (8,3) and det J at reference point xi."""
    N, dN = shape(xi)
    J = Xe.T @ dN                   # J[d, k] = dx_d / dxi_k
    det = np.linalg.det(J)
    G = dN @ np.linalg.inv(J)       # dN_a/dx_d = sum_k dN_a/dxi_k dxi_k/dx_d
    return N, G, det


def strain_matrix(G: np.ndarray) -> np.ndarray:
    """B (6 x 24): engineering strain of a displacement ordered (node, comp)."""
    B = np.zeros((6, 24))
    for a in range(8):
        gx, gy, gz = G[a]
        c = 3 * a
        B[0, c + 0] = gx
        B[1, c + 1] = gy
        B[2, c + 2] = gz
        B[3, c + 1], B[3, c + 2] = gz, gy
        B[4, c + 0], B[4, c + 2] = gz, gx
        B[5, c + 0], B[5, c + 1] = gy, gx
    return B


def ke_elastic(Xe: np.ndarray, C: np.ndarray) -> np.ndarray:
    K = np.zeros((24, 24))
    for xi, wq in quad_points():
        _, G, det = _grad_det(Xe, xi)
        B = strain_matrix(G)
        K += B.T @ C @ B * (det * wq)
    return K


def ke_scalar(Xe: np.ndarray, k: float) -> np.ndarray:
    K = np.zeros((8, 8))
    for xi, wq in quad_points():
        _, G, det = _grad_det(Xe, xi)
        K += k * (G @ G.T) * (det * wq)
    return K


def fe_body(Xe: np.ndarray, f: np.ndarray) -> np.ndarray:
    """Element load int f . phi_a (ncomp per node, node-major)."""
    out = np.zeros((8, len(f)))
    for xi, wq in quad_points():
        N, _, det = _grad_det(Xe, xi)
        out += np.outer(N, f) * (det * wq)
    return out.ravel()


def fe_top_traction(Xe: np.ndarray, g: np.ndarray) -> np.ndarray:
    """Element load of a traction g on the face zeta = +1 (2x2 Gauss)."""
    out = np.zeros((8, len(g)))
    for gy in GP:
        for gx in GP:
            xi = np.array([gx, gy, 1.0])
            N, dN = shape(xi)
            t1 = Xe.T @ dN[:, 0]
            t2 = Xe.T @ dN[:, 1]
            area = np.linalg.norm(np.cross(t1, t2))
            out += np.outer(N, g) * area
    return out.ravel()


def element_matrices(w, elems=None) -> np.ndarray:
    """K_e for the given elements (all by default): (n, 24, 24) or (n, 8, 8)."""
    X = node_xyz(w)
    elems = np.arange(w.n_elem) if elems is None else np.asarray(elems)
    en = elem_nodes(w, elems)
    nd = 8 * w.ncomp
    out = np.empty((len(elems), nd, nd))
    cache = {}
    for t, e in enumerate(elems):
        Xe = X[en[t]]
        if w.pde == 1:
            m = int(w.elem_mat[e])
            th = float(w.elem_angle[e]) if w.elem_angle is not None else 0.0
            tl = float(w.elem_tilt[e]) if w.elem_tilt is not None else 0.0
            key = (m, th, tl)
            if key not in cache:
                cache[key] = material_C(w.mats[m], th, tl)
            out[t] = ke_elastic(Xe, cache[key])
        else:
            out[t] = ke_scalar(Xe, float(w.elem_k[e]))
    return out


def elem_dofs(w, en: np.ndarray) -> np.ndarray:
    """Full DOF ids (n, 8*ncomp) of element node lists, node-major."""
    nc = w.ncomp
    return (en[:, :, None] * nc + np.arange(nc)[None, None, :]).reshape(len(en), -1)


# ---------------------------------------------------------------------------
# assembly (eqn:fe_matrix_system) with Dirichlet elimination
# ---------------------------------------------------------------------------

def assemble_full(w, Ke=None):
    """Full-DOF stiffness (all nodes, no BCs) as CSR, from element matrices."""
    if Ke is None:
        Ke = element_matrices(w)
    en = elem_nodes(w, np.arange(w.n_elem))
    dofs = elem_dofs(w, en)
    nd = dofs.shape[1]
    rows = np.repeat(dofs, nd, axis=1).ravel()
    cols = np.tile(dofs, (1, nd)).ravel()
    n = w.n_dof_full
    return sp.coo_matrix((Ke.ravel(), (rows, cols)), shape=(n, n)).tocsr()


def load_full(w) -> np.ndarray:
    """Full-DOF load vectors (n_dof_full, nrhs): body force + top tractions."""
    n, nc = w.n_dof_full, w.ncomp
    b = np.zeros((n, w.nrhs))
    X = node_xyz(w)
    if w.body is not None:
        en = elem_nodes(w, np.arange(w.n_elem))
        dofs = elem_dofs(w, en)
        f = w.body.reshape(w.n_elem, nc)
        for e in range(w.n_elem):
            if np.any(f[e] != 0):
                be = fe_body(X[en[e]], f[e])
                b[dofs[e], :] += be[:, None]
    if w.traction is not None:
        nx, ny, nz = w.ne
        g = w.traction.reshape(w.nrhs, nx * ny, nc)          # [rhs][face][comp]
        top = np.arange(nx * ny) + nx * ny * (nz - 1)
        en = elem_nodes(w, top)
        dofs = elem_dofs(w, en)
        for t in range(nx * ny):
            for r in range(w.nrhs):
                if np.any(g[r, t] != 0):
                    b[dofs[t], r] += fe_top_traction(X[en[t]], g[r, t])
    return b


def assemble_rows(w, free_rows):
    """Selected rows of the free-DOF system, each summed from the element
    matrices of the elements around its node (for sampled checks at sizes
    where a full assembly is too slow).  Returns (cols, vals, b) per row, cols
    in free numbering."""
    free = w.free_index()
    free_of_full = -np.ones(w.n_dof_full, dtype=np.int64)
    free_of_full[free] = np.arange(len(free))
    nc = w.ncomp
    nx, ny, nz = w.ne
    NX, NY = nx + 1, ny + 1
    out = []
    X = node_xyz(w)
    for fr in free_rows:
        full = int(free[fr])
        node, comp = divmod(full, nc)
        i, j, k = node % NX, (node // NX) % NY, node // (NX * NY)
        elems = [ex + nx * (ey + ny * ez)
                 for ez in (k - 1, k) for ey in (j - 1, j) for ex in (i - 1, i)
                 if 0 <= ex < nx and 0 <= ey < ny and 0 <= ez < nz]
        Ke = element_matrices(w, elems)
        en = elem_nodes(w, np.array(elems))
        dofs = elem_dofs(w, en)
        row = {}
        bval = 0.0
        for t, e in enumerate(elems):
            a = int(np.flatnonzero(en[t] == node)[0])
            li = a * nc + comp
            for lj, dj in enumerate(dofs[t]):
                fj = free_of_full[dj]
                if fj >= 0:
                    row[fj] = row.get(fj, 0.0) + Ke[t][li, lj]
            if w.body is not None:
                bval += fe_body(X[en[t]], w.body.reshape(w.n_elem, nc)[e])[li]
        if w.traction is not None:
            g = w.traction.reshape(w.nrhs, nx * ny, nc)
            for t, e in enumerate(elems):
                if e // (nx * ny) == nz - 1:
                    a = int(np.flatnonzero(en[t] == node)[0])
                    bval += fe_top_traction(X[en[t]], g[0, e % (nx * ny)])[a * nc + comp]
        cols = np.array(sorted(row))
        out.append((cols, np.array([row[c] for c in cols]), bval))
    return out


def assemble(w, Ke=None):
    """Free-DOF system (A, b, free) with homogeneous Dirichlet DOFs dropped."""
    Afull = assemble_full(w, Ke)
    free = w.free_index()
    A = Afull[free][:, free].tocsr()
    b = load_full(w)[free]
    return A, b, free
