"""Workload generator: seeded, synthetic inputs shaped like the paper's problems.

Conventions shared by every consumer (they are *interface* conventions, not
arithmetic of the method):

* Tensor grid with ``ne = (nx, ny, nz)`` hexahedral elements and node
  coordinates ``xn[a]`` (length ``ne[a] + 1``) per axis.
* Node ``(i, j, k)`` has linear id ``i + (nx+1) * (j + (ny+1) * k)`` (x fastest);
  element ``(ex, ey, ez)`` has id ``ex + nx * (ey + ny * ez)``.
* Optional ramp map (``map_kind == 1``, ``map_par = (x0, x1, angle)``): the
  physical node position is ``(x, y, z + r(x))`` with ``r`` continuous and
  piecewise linear, slope ``tan(angle)`` on ``[x0, x1]`` and flat elsewhere.
* ``pde == 1`` is linear elasticity (3 components per node, component fastest);
  ``pde == 0`` is scalar diffusion (1 component).
* Materials are 9 engineering constants ``(E1, E2, E3, G12, G13, G23, nu12,
  nu13, nu23)`` in MPa; lengths are in mm (the paper's units).
* ``elem_angle`` is the in-plane fibre angle (radians, counter-clockwise about
  +z seen from +z); ``elem_tilt`` (radians) tilts the laminate about y so the
  material x axis becomes ``(cos t, 0, sin t)``.
* ``dirichlet`` is a per (node, component) 0/1 mask of homogeneous Dirichlet
  DOFs; ``body`` is a constant body force per element (``ncomp`` values);
  ``traction`` is a constant traction per top-face element (``nx*ny`` faces,
  x fastest) per component per right-hand side.
* Subdomains are a tensor product of per-axis element cuts; subdomain
  ``(p, q, r)`` has id ``p + Px * (q + Py * r)``.

Paper constants (Section 5, material properties paragraph): plies are
orthotropic with E11 = 162 GPa, E22 = E33 = 10 GPa, G12 = G13 = 5.2 GPa,
G23 = 3.5 GPa, nu12 = nu13 = 0.35, nu23 = 0.5, thickness 0.23 mm; resin
interlayers are isotropic with E = 10 GPa, nu = 0.35, thickness 0.02 mm.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

# (E1, E2, E3, G12, G13, G23, nu12, nu13, nu23) in MPa.
PLY_CONSTS = np.array([162000.0, 10000.0, 10000.0, 5200.0, 5200.0, 3500.0,
                       0.35, 0.35, 0.5])


def iso_consts(E: float, nu: float) -> np.ndarray:
    """Isotropic material written in the 9-constant orthotropic form."""
    G = E / (2.0 * (1.0 + nu))
    return np.array([E, E, E, G, G, G, nu, nu, nu], dtype=np.float64)


RESIN_CONSTS = iso_consts(10000.0, 0.35)
PLY_T = 0.23
RESIN_T = 0.02


@dataclasses.dataclass
class Workload:
    name: str
    pde: int                      # 0 scalar diffusion, 1 elasticity
    ne: Tuple[int, int, int]
    xn: List[np.ndarray]          # node coordinates per axis
    map_kind: int = 0
    map_par: Optional[np.ndarray] = None
    mats: Optional[np.ndarray] = None       # (n_mat, 9) float64
    elem_mat: Optional[np.ndarray] = None   # int32 (n_elem,)
    elem_angle: Optional[np.ndarray] = None  # float64 (n_elem,)
    elem_tilt: Optional[np.ndarray] = None   # float64 (n_elem,)
    elem_k: Optional[np.ndarray] = None      # float64 (n_elem,) scalar pde
    dirichlet: Optional[np.ndarray] = None   # uint8 (n_node*ncomp,)
    body: Optional[np.ndarray] = None        # float64 (n_elem*ncomp,)
    nrhs: int = 1
    traction: Optional[np.ndarray] = None    # float64 (nx*ny*ncomp*nrhs,)
    nparts: Tuple[int, int, int] = (1, 1, 1)
    cuts: Optional[List[np.ndarray]] = None
    overlap: int = 1
    nev: int = 0
    threshold: float = 0.0
    nev_max: int = 0
    seed: Optional[int] = None
    pou: str = "standard"                    # partition of unity: "standard" or "sarkis"
    meta: dict = dataclasses.field(default_factory=dict)

    # --- sizes only -----------------------------------------------------
    @property
    def ncomp(self) -> int:
        return 3 if self.pde == 1 else 1

    @property
    def nn(self) -> Tuple[int, int, int]:
        return (self.ne[0] + 1, self.ne[1] + 1, self.ne[2] + 1)

    @property
    def n_node(self) -> int:
        a, b, c = self.nn
        return a * b * c

    @property
    def n_elem(self) -> int:
        return self.ne[0] * self.ne[1] * self.ne[2]

    @property
    def n_dof_full(self) -> int:
        return self.n_node * self.ncomp

    @property
    def n_free(self) -> int:
        return int(self.n_dof_full - int(self.dirichlet.sum()))

    @property
    def n_sub(self) -> int:
        return int(np.prod(self.nparts))

    def free_index(self) -> np.ndarray:
        """Full DOF id (node*ncomp + comp) of every free DOF, in free order."""
        return np.flatnonzero(self.dirichlet == 0).astype(np.int64)


# ---------------------------------------------------------------------------
# building blocks
# ---------------------------------------------------------------------------

def _layers_to_z(layers: Sequence[Tuple[str, float, int, float]]):
    """layers: (kind 'ply'|'resin', angle_deg, n_elements, thickness)."""
    zs = [0.0]
    zmat, zang = [], []
    for kind, ang, nel, thick in layers:
        h = thick / nel
        for _ in range(nel):
            zs.append(zs[-1] + h)
            zmat.append(0 if kind == "ply" else 1)
            zang.append(math.radians(ang) if kind == "ply" else 0.0)
    return np.array(zs), np.array(zmat, dtype=np.int32), np.array(zang)


def uniform_cuts(n: int, parts: int) -> np.ndarray:
    """Near-uniform cuts floor(p*n/P)."""
    return np.array([(p * n) // parts for p in range(parts + 1)], dtype=np.int32)


def uneven_cuts(n: int, parts: int, rng: np.random.Generator,
                lo: float = 0.7, hi: float = 1.3, min_w: int = 2) -> np.ndarray:
    """Per-axis widths proportional to U(lo, hi), cumulatively rounded."""
    if parts == 1:
        return np.array([0, n], dtype=np.int32)
    for _ in range(1000):
        w = rng.uniform(lo, hi, size=parts)
        c = np.concatenate([[0.0], np.cumsum(w)]) / w.sum() * n
        cuts = np.rint(c).astype(np.int32)
        cuts[0], cuts[-1] = 0, n
        if np.all(np.diff(cuts) >= min_w):
            return cuts
    raise ValueError("could not draw uneven cuts")


def _elem_grid(ne):
    nx, ny, nz = ne
    ez, ey, ex = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx),
                             indexing="ij")
    return ex.ravel(), ey.ravel(), ez.ravel()


def _node_grid(nn):
    a, b, c = nn
    k, j, i = np.meshgrid(np.arange(c), np.arange(b), np.arange(a), indexing="ij")
    return i.ravel(), j.ravel(), k.ravel()


def laminate_plate(ne_xy: Tuple[int, int], size_xy: Tuple[float, float],
                   layers, nparts, cuts=None, overlap=1, nev=10, threshold=0.0,
                   nev_max=0, clamp_x0=True, body=(0.0, 0.0, -1.0),
                   traction=None, nrhs=1, name="laminate", seed=None,
                   resin=RESIN_CONSTS, ramp=None, meta=None) -> Workload:
    """Laminate box: plies + resin interlayers stacked in z, clamped at x=0."""
    zs, zmat, zang = _layers_to_z(layers)
    nx, ny = ne_xy
    nz = len(zmat)
    ne = (nx, ny, nz)
    xn = [np.linspace(0.0, size_xy[0], nx + 1), np.linspace(0.0, size_xy[1], ny + 1), zs]
    ex, ey, ez = _elem_grid(ne)
    elem_mat = zmat[ez].astype(np.int32)
    elem_angle = zang[ez].astype(np.float64)
    w = Workload(name=name, pde=1, ne=ne, xn=xn, mats=np.stack([PLY_CONSTS, resin]),
                 elem_mat=elem_mat, elem_angle=elem_angle, seed=seed,
                 meta=dict(meta or {}))
    if ramp is not None:
        x0, x1, ang = ramp
        w.map_kind = 1
        w.map_par = np.array([x0, x1, ang], dtype=np.float64)
        # fibres follow the local slope of the ramped laminate
        xc = 0.5 * (xn[0][ex] + xn[0][ex + 1])
        w.elem_tilt = np.where((xc > x0) & (xc < x1), ang, 0.0).astype(np.float64)
    nnx, nny, nnz = w.nn
    ni, nj, nk = _node_grid(w.nn)
    dmask = np.zeros((w.n_node, 3), dtype=np.uint8)
    if clamp_x0:
        dmask[ni == 0, :] = 1
    w.dirichlet = dmask.ravel()
    if body is not None:
        w.body = np.tile(np.asarray(body, dtype=np.float64), w.n_elem)
    if traction is not None:
        w.nrhs = nrhs
        w.traction = np.asarray(traction, dtype=np.float64).ravel()
    w.nparts = tuple(int(p) for p in nparts)
    w.cuts = [np.asarray(c, dtype=np.int32) for c in cuts] if cuts is not None else \
        [uniform_cuts(ne[a], nparts[a]) for a in range(3)]
    w.overlap, w.nev, w.threshold, w.nev_max = overlap, nev, threshold, nev_max
    return w


def diffusion_box(ne, k: np.ndarray, nparts, cuts=None, overlap=1, nev=0,
                  threshold=0.15, nev_max=32, dirichlet_faces=("x0", "x1"),
                  f=1.0, name="diffusion", seed=None, h=1.0, meta=None) -> Workload:
    """Scalar -div(k grad u) = f on unit cells, homogeneous Dirichlet faces."""
    ne = tuple(int(v) for v in ne)
    xn = [np.arange(ne[a] + 1, dtype=np.float64) * h for a in range(3)]
    w = Workload(name=name, pde=0, ne=ne, xn=xn, elem_k=np.asarray(k, np.float64).ravel(),
                 seed=seed, meta=dict(meta or {}))
    ni, nj, nk = _node_grid(w.nn)
    d = np.zeros(w.n_node, dtype=np.uint8)
    for face in dirichlet_faces:
        ax = "xyz".index(face[0])
        idx = (ni, nj, nk)[ax]
        d[idx == (0 if face[1] == "0" else ne[ax])] = 1
    w.dirichlet = d
    w.body = np.full(w.n_elem, float(f))
    w.nparts = tuple(int(p) for p in nparts)
    w.cuts = [np.asarray(c, dtype=np.int32) for c in cuts] if cuts is not None else \
        [uniform_cuts(ne[a], nparts[a]) for a in range(3)]
    w.overlap, w.nev, w.threshold, w.nev_max = overlap, nev, threshold, nev_max
    return w


def gaussian_random_field(shape, corr_len: float, sigma: float,
                          rng: np.random.Generator) -> Tuple[np.ndarray, float]:
    """Stationary field with covariance sigma^2 exp(-r / corr_len) (r in cells).

    Circulant embedding on a periodic grid twice the size per axis; negative
    embedding eigenvalues are clipped and the clipped fraction is returned.
    """
    big = tuple(2 * s for s in shape)
    axes = [np.minimum(np.arange(n), n - np.arange(n)).astype(np.float64) for n in big]
    dx, dy, dz = np.meshgrid(*axes, indexing="ij")
    r = np.sqrt(dx * dx + dy * dy + dz * dz)
    cov = sigma * sigma * np.exp(-r / corr_len)
    lam = np.fft.fftn(cov).real
    neg = float(-lam[lam < 0].sum() / np.abs(lam).sum())
    lam = np.clip(lam, 0.0, None)
    m = lam.size
    xi = rng.standard_normal(big) + 1j * rng.standard_normal(big)
    z = np.fft.fftn(np.sqrt(lam / m) * xi)
    field = z.real[: shape[0], : shape[1], : shape[2]]
    return np.ascontiguousarray(field), neg


def spe10_like(ne=(60, 220, 85), nparts=(8, 8, 4), overlap=2, threshold=0.15,
               nev_max=32, seed=2, sigma=2.0, corr_len=4.0, channel_frac=0.2,
               contrast=1e6, name="spe10_like") -> Workload:
    """Synthetic stand-in for the SPE10 permeability (the dataset itself is
    not available): log-normal background plus channelised layers."""
    rng = np.random.default_rng(seed)
    g, neg = gaussian_random_field(ne, corr_len, sigma, rng)   # indexed [x, y, z]
    k = np.exp(g)
    nx, ny, nz = ne
    n_ch = int(round(channel_frac * nz))
    layers = rng.choice(nz, size=n_ch, replace=False)
    xc = np.arange(nx) + 0.5
    yc = np.arange(ny) + 0.5
    for L in sorted(layers):
        lay = np.ones((nx, ny))
        for _ in range(4):
            x0 = rng.uniform(0, nx)
            A = rng.uniform(2, 6)
            Lam = rng.uniform(40, 110)
            ph = rng.uniform(0, 2 * np.pi)
            cent = x0 + A * np.sin(2 * np.pi * yc / Lam + ph)
            inside = np.abs(xc[:, None] - cent[None, :]) <= 1.5
            lay[inside] = contrast
        k[:, :, L] = lay
    # element id is x fastest: transpose [x,y,z] -> ravel over (z,y,x)
    kel = np.transpose(k, (2, 1, 0)).ravel()
    return diffusion_box(ne, kel, nparts, overlap=overlap, threshold=threshold,
                         nev_max=nev_max, name=name, seed=seed,
                         meta=dict(clipped_embedding_mass=neg,
                                   channel_layers=sorted(int(v) for v in layers)))


# ---------------------------------------------------------------------------
# the named configurations
# ---------------------------------------------------------------------------

def config_c1() -> Workload:
    """16x16x8 Q1 laminate: [0, R, 90, R, 45, R, -45, -45] bottom to top, the
    top ply split in two elements; clamp x=0; body force (0,0,-1); 2x2x1
    subdomains, overlap 1, 10 eigenvectors per subdomain."""
    layers = [("ply", 0, 1, PLY_T), ("resin", 0, 1, RESIN_T),
              ("ply", 90, 1, PLY_T), ("resin", 0, 1, RESIN_T),
              ("ply", 45, 1, PLY_T), ("resin", 0, 1, RESIN_T),
              ("ply", -45, 2, PLY_T)]
    return laminate_plate((16, 16), (16.0, 16.0), layers, nparts=(2, 2, 1),
                          overlap=1, nev=10, name="c1_laminate_16x16x8")


def config_c2(**kw) -> Workload:
    """SPE10-shaped 60x220x85 high-contrast diffusion, 8x8x4 subdomains,
    overlap 2, threshold 0.15 (cap 32)."""
    return spe10_like(**kw)


def _random_layup(n_ply, rng, elems_per_ply, total_z):
    angles = rng.choice([0.0, 90.0, 45.0, -45.0], size=n_ply)
    layers = []
    used = n_ply * elems_per_ply + (n_ply - 1)
    extra = total_z - used
    for p in range(n_ply):
        ne = elems_per_ply + (extra if p == n_ply - 1 else 0)
        layers.append(("ply", float(angles[p]), ne, PLY_T))
        if p != n_ply - 1:
            layers.append(("resin", 0.0, 1, RESIN_T))
    return layers, angles


def config_c3(seed: int = 3) -> Workload:
    """200x40x48 Q1 laminate (12 random plies) with 16x4x4 uneven subdomains."""
    rng = np.random.default_rng(seed)
    layers, angles = _random_layup(12, rng, 3, 48)
    nparts = (16, 4, 4)
    nz = sum(l[2] for l in layers)
    cuts = [uneven_cuts(200, 16, rng), uneven_cuts(40, 4, rng), uneven_cuts(nz, 4, rng)]
    return laminate_plate((200, 40), (100.0, 20.0), layers, nparts=nparts, cuts=cuts,
                          overlap=1, nev=12, name="c3_laminate_200x40x48", seed=seed,
                          meta=dict(angles=[float(a) for a in angles]))


def _c4_operator(size_dofs: float, n_ply: int, rng: np.random.Generator, h: float = 0.5,
                 aspect: float = 5.0, target_nj: float = 5000.0, name: str = "c4") -> Workload:
    """One laminate of the serving catalogue: c3's element rule (3 elements
    per ply, 1 per resin interlayer) at in-plane size h, in-plane aspect
    `aspect`:1, about `size_dofs` DOFs, near-cubic subdomains of about
    `target_nj` local DOFs, overlap 1, 12 eigenvectors; clamped at x = 0 and
    loaded only by the tractions of each request (no body force)."""
    nz = 4 * n_ply - 1
    ny = max(2, int(round(math.sqrt(size_dofs / (3.0 * (nz + 1) * aspect)))) - 1)
    nx = max(2, int(round(aspect * (ny + 1))) - 1)
    layers, angles = _random_layup(n_ply, rng, 3, nz)
    ne = (nx, ny, nz)
    n_sub = max(1.0, size_dofs / target_nj)
    side = (nx * ny * nz / n_sub) ** (1.0 / 3.0)
    nparts = tuple(max(1, min(ne[a] // 3, int(round(ne[a] / side)))) for a in range(3))
    return laminate_plate((nx, ny), (nx * h, ny * h), layers, nparts=nparts, overlap=1, nev=12,
                          body=None, name=name, meta=dict(angles=[float(a) for a in angles]))


def config_c4_catalogue(seed: int = 4, sizes=(0.2e6, 0.5e6, 1.0e6, 2.0e6), layups: int = 4,
                        ply_range=(8, 24)) -> List[Workload]:
    """Serving catalogue: len(sizes) x `layups` laminate operators, 8-24 random
    plies each (angles iid from {0, 90, 45, -45})."""
    rng = np.random.default_rng(seed)
    cat = []
    for si, S in enumerate(sizes):
        for li in range(layups):
            n_ply = int(rng.integers(ply_range[0], ply_range[1] + 1))
            cat.append(_c4_operator(S, n_ply, rng, name=f"c4_op{si}{li}_{int(S / 1e3)}k_{n_ply}ply"))
    return cat


def patch_tractions(w: Workload, k: int, rng: np.random.Generator, sigma: float = 0.01,
                    side=(0.1, 0.5)) -> np.ndarray:
    """k load cases: each a uniform traction, components ~ N(0, sigma) MPa, on
    an axis-aligned patch of the top face whose sides are U(side) x the face's
    length along that axis.  Layout [rhs][face = ex + nx * ey][comp]."""
    nx, ny = w.ne[0], w.ne[1]
    xc = 0.5 * (w.xn[0][:-1] + w.xn[0][1:])
    yc = 0.5 * (w.xn[1][:-1] + w.xn[1][1:])
    Lx, Ly = w.xn[0][-1] - w.xn[0][0], w.xn[1][-1] - w.xn[1][0]
    out = np.zeros((k, ny, nx, 3))
    for r in range(k):
        ax, ay = rng.uniform(*side) * Lx, rng.uniform(*side) * Ly
        x0 = w.xn[0][0] + rng.uniform(0.0, Lx - ax)
        y0 = w.xn[1][0] + rng.uniform(0.0, Ly - ay)
        g = rng.normal(0.0, sigma, size=3)
        mx = (xc >= x0) & (xc <= x0 + ax)
        my = (yc >= y0) & (yc <= y0 + ay)
        out[r][np.ix_(my, mx)] = g
    return out.reshape(-1)


def c4_requests(n_ops: int, n_req: int = 1000, rate: float = 20.0, max_rhs: int = 16,
                seed: int = 4) -> List[dict]:
    """Poisson arrivals (mean `rate` per second): arrival time, operator index
    (uniform) and number of right-hand sides U{1..max_rhs}; each request's
    tractions come from patch_tractions with the generator seeded by
    (seed, request index)."""
    rng = np.random.default_rng([seed, 1])
    t = np.cumsum(rng.exponential(1.0 / rate, size=n_req))
    ops = rng.integers(0, n_ops, size=n_req)
    ks = rng.integers(1, max_rhs + 1, size=n_req)
    return [dict(t=float(t[i]), op=int(ops[i]), k=int(ks[i]), seed=(seed, 2, i)) for i in range(n_req)]


EXAMPLE1_STACK = [-45.0, 45.0, 0.0, 90.0, 45.0, -45.0, -45.0, 45.0, 90.0, 0.0, 45.0, -45.0]


def example1b_plate(nparts, nxy=(35, 7), threshold=0.15, nev_max=32) -> Workload:
    """The flat plate of the paper's Example 1 (Section 5): 100 mm x 20 mm, the
    12-ply stacking sequence of eqn:stackingSeq_Example01 with 11 resin
    interfaces, 2 elements per ply and 1 per interface through the thickness,
    clamped at x = 0, uniform pressure 0.01 MPa on the top face.  Q1 elements
    (35 x 7 in plane: 30,240 free DOFs, near the 30,000 of the Example 1b
    table); GenEO by threshold."""
    layers = []
    for p, a in enumerate(EXAMPLE1_STACK):
        layers.append(("ply", a, 2, PLY_T))
        if p != len(EXAMPLE1_STACK) - 1:
            layers.append(("resin", 0.0, 1, RESIN_T))
    nx, ny = nxy
    trac = np.tile(np.array([0.0, 0.0, -0.01]), nx * ny)
    return laminate_plate((nx, ny), (100.0, 20.0), layers, nparts=nparts, overlap=1, nev=0,
                          threshold=threshold, nev_max=nev_max, body=None, traction=trac, nrhs=1,
                          name=f"example1b_{nparts[0]}x{nparts[1]}x{nparts[2]}")


def contrast_box(contrast: float, nparts, ne=(32, 32, 32), seed: int = 12, threshold=0.15,
                 nev_max=32) -> Workload:
    """Scalar diffusion on a unit-cell box, u = 0 on the x faces, f = 1: k = 1
    with every fifth z-layer crossed by three channels (3 cells wide, along y)
    of conductivity `contrast` (the same channels for every contrast)."""
    rng = np.random.default_rng(seed)
    k = np.ones(ne)
    for L in range(2, ne[2], 5):
        for _ in range(3):
            x0 = rng.uniform(2, ne[0] - 2)
            k[np.abs(np.arange(ne[0]) + 0.5 - x0) <= 1.5, :, L] = contrast
    kel = np.transpose(k, (2, 1, 0)).ravel()
    return diffusion_box(ne, kel, nparts, overlap=1, threshold=threshold, nev_max=nev_max,
                         name=f"contrast_{contrast:g}_{nparts[0]}x{nparts[1]}x{nparts[2]}", seed=seed)


def config_c5() -> Workload:
    """384x72x71 ramped laminate, 24 plies x 2 elements + 23 resin, resin
    contrast 1e3, top pressure 0.01 MPa, 32x12x4 subdomains."""
    layers = []
    for p in range(24):
        layers.append(("ply", [0, 90, 45, -45][p % 4], 2, PLY_T))
        if p != 23:
            layers.append(("resin", 0.0, 1, RESIN_T))
    nx, ny = 384, 72
    trac = np.tile(np.array([0.0, 0.0, -0.01]), nx * ny)
    return laminate_plate((nx, ny), (192.0, 36.0), layers, nparts=(32, 12, 4),
                          overlap=1, nev=12, body=None, traction=trac, nrhs=1,
                          resin=iso_consts(162.0, 0.35),
                          ramp=(64.0, 128.0, math.radians(10.0)),
                          name="c5_ramp_384x72x71")


def small_case(kind: str = "laminate", seed: int = 0, **kw) -> Workload:
    """Small versions of the configurations for tests (oracle runs in seconds)."""
    rng = np.random.default_rng(seed)
    if kind == "laminate":
        nx, ny = kw.get("nxy", (8, 6))
        n_ply = kw.get("n_ply", 3)
        angles = kw.get("angles") or [float(a) for a in rng.choice([0, 90, 45, -45], n_ply)]
        layers = []
        for p, a in enumerate(angles):
            layers.append(("ply", a, kw.get("elems_per_ply", 1), PLY_T))
            if p != len(angles) - 1:
                layers.append(("resin", 0.0, 1, RESIN_T))
        nparts = kw.get("nparts", (2, 2, 1))
        nz = sum(l[2] for l in layers)
        ne = (nx, ny, nz)
        cuts = kw.get("cuts")
        if cuts is None and kw.get("uneven", False):
            cuts = [uneven_cuts(ne[a], nparts[a], rng) for a in range(3)]
        return laminate_plate((nx, ny), kw.get("size", (float(nx), float(ny))), layers,
                              nparts=nparts, cuts=cuts, overlap=kw.get("overlap", 1),
                              nev=kw.get("nev", 8), threshold=kw.get("threshold", 0.0),
                              nev_max=kw.get("nev_max", 0),
                              traction=kw.get("traction"), nrhs=kw.get("nrhs", 1),
                              body=kw.get("body", (0.0, 0.0, -1.0)),
                              ramp=kw.get("ramp"), name=f"small_laminate_s{seed}",
                              seed=seed)
    if kind == "diffusion":
        ne = kw.get("ne", (10, 8, 6))
        contrast = kw.get("contrast", 1e6)
        g, _ = gaussian_random_field(ne, 2.0, 2.0, rng)
        k = np.exp(g)
        if kw.get("channels", True):
            for L in rng.choice(ne[2], size=max(1, ne[2] // 5), replace=False):
                xcen = rng.uniform(0, ne[0])
                k[:, :, L] = 1.0
                k[np.abs(np.arange(ne[0]) + 0.5 - xcen) <= 1.5, :, L] = contrast
        kel = np.transpose(k, (2, 1, 0)).ravel()
        return diffusion_box(ne, kel, kw.get("nparts", (2, 2, 2)), overlap=kw.get("overlap", 1),
                             nev=kw.get("nev", 0), threshold=kw.get("threshold", 0.15),
                             nev_max=kw.get("nev_max", 16),
                             dirichlet_faces=kw.get("dirichlet_faces", ("x0", "x1")),
                             name=f"small_diffusion_s{seed}", seed=seed)
    raise ValueError(kind)
