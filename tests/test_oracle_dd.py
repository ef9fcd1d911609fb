"""Pins of the oracle's decomposition and partition of unity (Section 3.2)."""
import numpy as np
import pytest

from oracle import dd
from workloads import generate as gen


CASES = [
    ("laminate", dict(nxy=(8, 6), n_ply=3, nparts=(2, 2, 1), overlap=1)),
    ("laminate", dict(nxy=(9, 7), n_ply=3, nparts=(3, 2, 2), overlap=1, uneven=True)),
    ("diffusion", dict(ne=(10, 8, 6), nparts=(2, 2, 2), overlap=2)),
    ("diffusion", dict(ne=(12, 9, 7), nparts=(3, 3, 2), overlap=1)),
]


@pytest.mark.parametrize("pou", ["standard", "sarkis"])
@pytest.mark.parametrize("kind,kw", CASES)
def test_partition_of_unity_sums_to_one(kind, kw, pou):
    w = gen.small_case(kind, seed=5, **kw)
    w.pou = pou
    d = dd.Decomposition(w)
    v = np.random.default_rng(0).standard_normal(w.n_free)
    assert np.max(np.abs(d.pou_sum(v) - v)) <= 4 * np.finfo(float).eps * np.max(np.abs(v))
    assert d.count.min() >= 1 and d.count.max() <= 8


@pytest.mark.parametrize("pou", ["standard", "sarkis"])
@pytest.mark.parametrize("kind,kw", CASES)
def test_pou_is_identity_off_the_overlap(kind, kw, pou):
    w = gen.small_case(kind, seed=6, **kw)
    w.pou = pou
    d = dd.Decomposition(w)
    for j in range(d.n_sub):
        # nodes all of whose adjacent elements are in Omega_j but not in Omega_j^o
        private = d.E[j] & ~d.E_ov[j]
        outside = np.zeros(w.n_node, bool)
        outside[d.en[~private].ravel()] = True
        touched = np.zeros(w.n_node, bool)
        touched[d.en[private].ravel()] = True
        nodes = np.flatnonzero(touched & ~outside)
        dofs = d._free_dofs(nodes)
        pos = np.searchsorted(d.Ibar[j], dofs)
        assert np.all(d.X[j][pos] == 1.0)
        # zero on Ibar_j \ I_j (the subdomain boundary)
        rest = np.setdiff1d(d.Ibar[j], d.I[j])
        assert np.all(d.X[j][np.searchsorted(d.Ibar[j], rest)] == 0.0)


def _box_count(lo, hi, n):
    # nodes of the element box [lo,hi): lo..hi ; interior-or-global-boundary nodes
    closure = hi - lo + 1
    first = 0 if lo == 0 else lo + 1
    last = n if hi == n else hi - 1
    return closure, max(0, last - first + 1)


@pytest.mark.parametrize("kind,kw", CASES)
def test_index_set_sizes_against_box_counts(kind, kw):
    w = gen.small_case(kind, seed=7, **kw)
    d = dd.Decomposition(w)
    boxes = dd.subdomain_boxes(w)
    O = w.overlap
    nc = w.ncomp
    for j, (lo, hi) in enumerate(boxes):
        cl, inn = 1, 1
        for a in range(3):
            c, i = _box_count(max(0, lo[a] - O), min(w.ne[a], hi[a] + O), w.ne[a])
            cl *= c
            inn *= i
        # subtract Dirichlet DOFs counted by brute force on the node boxes
        assert len(d.Ibar[j]) <= cl * nc and len(d.I[j]) <= inn * nc
        if w.pde == 1:      # clamp x=0 removes one node plane when the box touches it
            elo = max(0, lo[0] - O)
            ny_cl = min(w.ne[1], hi[1] + O) - max(0, lo[1] - O) + 1
            nz_cl = min(w.ne[2], hi[2] + O) - max(0, lo[2] - O) + 1
            if elo == 0:
                cl -= ny_cl * nz_cl
                _, iy = _box_count(max(0, lo[1] - O), min(w.ne[1], hi[1] + O), w.ne[1])
                _, iz = _box_count(max(0, lo[2] - O), min(w.ne[2], hi[2] + O), w.ne[2])
                inn -= iy * iz
            assert len(d.Ibar[j]) == cl * 3
            assert len(d.I[j]) == inn * 3


def test_zero_overlap_rejected():
    w = gen.small_case("laminate", seed=1, nxy=(8, 6), n_ply=2, overlap=0)
    with pytest.raises(ValueError):
        dd.Decomposition(w)


@pytest.mark.parametrize("overlap", [1, 2, 3])
def test_sarkis_pou_ramps_linearly_across_the_overlap(overlap):
    """Two subdomains split at x = c with overlap O: the left one spans elements
    [0, c + O), the right one [c - O, n), so at node index i of the overlap the
    distances to the artificial boundaries are c + O - i and i - (c - O), and the
    smooth PoU is their ratio to the sum 2 O (a linear ramp from 1 to 0); the
    standard PoU is 1/2 on the same nodes."""
    n, c = 12, 6
    w = gen.diffusion_box((n, 3, 2), np.ones(n * 3 * 2), (2, 1, 1), cuts=[np.array([0, c, n]),
                          np.array([0, 3]), np.array([0, 2])], overlap=overlap, threshold=0.15,
                          nev_max=4, dirichlet_faces=("x0",))
    w.pou = "sarkis"
    d = dd.Decomposition(w)
    full = w.free_index()
    for j, left in ((0, True), (1, False)):
        xi = (full[d.Ibar[j]] // w.ncomp) % (n + 1)
        for i in range(c - overlap + 1, c + overlap):
            expect = (c + overlap - i) / (2 * overlap) if left else (i - (c - overlap)) / (2 * overlap)
            assert np.allclose(d.X[j][xi == i], expect, rtol=0, atol=1e-15), (j, i)
        far = xi <= c - overlap if left else xi >= c + overlap
        inner = np.isin(d.Ibar[j], d.I[j])
        assert np.all(d.X[j][far & inner] == 1.0)
    w.pou = "standard"
    d0 = dd.Decomposition(w)
    xi = (full[d0.Ibar[0]] // w.ncomp) % (n + 1)
    mid = (xi > c - overlap) & (xi < c + overlap)
    assert np.all(d0.X[0][mid] == 0.5)
