"""Oracle: overlapping decomposition, index sets and partition of unity.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 3.1: non-overlapping subdomains Omega'_j (here boxes between per-axis
element cuts) are extended by O layers of elements to Omega_j;
V_h(Omega_j) is the restriction of V_h to Omega_j and V_{h,0}(Omega_j) the FE
functions whose support lies in Omega_j.  Section 3.2 defines the overlap
Omega_j^o (points of Omega_j in at least one other subdomain) and the partition
of unity; Section 3.3.1 builds the standard PoU as a diagonal X^(j) holding
one over the number of subdomains that contain the DOF, zero on the
subdomain boundary.

Readings:
* Omega_j is the element box extended by O elements per side, clipped to the
  mesh (structured overlapping grid);
* Omega_j^o is the set of elements of Omega_j that also belong to another
  Omega_j';
* the DOFs of V_h(Omega_j) ("Ibar_j") are the free DOFs at nodes of elements
  of Omega_j; those of V_{h,0}(Omega_j) ("I_j") are the free DOFs at nodes
  all of whose adjacent elements lie in Omega_j;
* the PoU counts, for each DOF, the subdomains whose I_j contains it (the
  count over closures would break the partition-of-unity identity);
* the smoother PoU the paper also provides (Sarkis) weights each subdomain by
  the distance to its artificial boundary (see ``_sarkis_pou``).

Every set is computed by brute force from these definitions (membership
counts over all subdomains), not from box arithmetic.

Pins (tests/test_oracle_dd.py): sum_j R_j^T X_j 1 = 1, X_j = 1 off the overlap,
1 <= c(i) <= 8, |I_j| and |Ibar_j| against closed-form box counts.
"""
from __future__ import annotations

import numpy as np

from .fem import elem_nodes


def subdomain_boxes(w):
    """Non-overlapping element boxes [lo, hi) per axis for every subdomain."""
    P = w.nparts
    boxes = []
    for r in range(P[2]):
        for q in range(P[1]):
            for p in range(P[0]):
                lo = [int(w.cuts[0][p]), int(w.cuts[1][q]), int(w.cuts[2][r])]
                hi = [int(w.cuts[0][p + 1]), int(w.cuts[1][q + 1]), int(w.cuts[2][r + 1])]
                boxes.append((lo, hi))
    return boxes


def _elem_ijk(w):
    nx, ny, _ = w.ne
    e = np.arange(w.n_elem)
    return e % nx, (e // nx) % ny, e // (nx * ny)


class Decomposition:
    """All index sets of the overlapping decomposition (free-DOF numbering)."""

    def __init__(self, w):
        self.w = w
        O = w.overlap
        ex, ey, ez = _elem_ijk(w)
        E = []
        for lo, hi in subdomain_boxes(w):
            elo = [max(0, lo[a] - O) for a in range(3)]
            ehi = [min(w.ne[a], hi[a] + O) for a in range(3)]
            m = ((ex >= elo[0]) & (ex < ehi[0]) & (ey >= elo[1]) & (ey < ehi[1])
                 & (ez >= elo[2]) & (ez < ehi[2]))
            E.append(m)
        self.E = E                                   # element masks of Omega_j
        count = np.sum(np.stack(E), axis=0)
        self.E_ov = [m & (count >= 2) for m in E]    # elements of Omega_j^o
        # node -> adjacent elements
        en = elem_nodes(w, np.arange(w.n_elem))
        self.en = en
        nn = w.n_node
        nc = w.ncomp
        free_of_full = -np.ones(w.n_dof_full, dtype=np.int64)
        free_of_full[w.free_index()] = np.arange(w.n_free)
        self.free_of_full = free_of_full
        self.Ibar, self.I = [], []
        for m in E:
            touched = np.zeros(nn, dtype=bool)
            touched[en[m].ravel()] = True
            # nodes with an adjacent element outside Omega_j
            outside = np.zeros(nn, dtype=bool)
            outside[en[~m].ravel()] = True
            inner = touched & ~outside
            self.Ibar.append(self._free_dofs(np.flatnonzero(touched)))
            self.I.append(self._free_dofs(np.flatnonzero(inner)))
        cnt = np.zeros(w.n_free, dtype=np.int64)
        for I in self.I:
            cnt[I] += 1
        self.count = cnt
        if np.any(cnt == 0):
            raise ValueError("some free DOF lies in no V_h0(Omega_j): overlap too small")
        self.pou = getattr(w, "pou", "standard")
        if self.pou == "standard":
            # PoU diagonal on Ibar_j: 1/c on I_j, 0 on Ibar_j \ I_j
            self.X = []
            for Ib, I in zip(self.Ibar, self.I):
                x = np.zeros(len(Ib))
                pos = np.searchsorted(Ib, I)
                x[pos] = 1.0 / cnt[I]
                self.X.append(x)
        elif self.pou == "sarkis":
            self.X = self._sarkis_pou()
        else:
            raise ValueError(f"unknown partition of unity {self.pou!r}")

    def _sarkis_pou(self):
        """Smooth PoU (Section 3.2, the Sarkis variant named after def:pou, and
        Section 3.3.1): the weight of subdomain j at a DOF of V_h0(Omega_j) is
        the distance of its node to the artificial boundary of Omega_j, and
        X_j = w_j / sum_k w_k.  Reading: the artificial boundary is the set of
        nodes of Omega_j that touch an element outside Omega_j (Ibar_j minus
        I_j), distances are measured on the node lattice as the largest index
        difference over the three axes (one element layer = 1), and a
        subdomain without artificial boundary (a single subdomain) has weight 1.
        Computed by brute force over all pairs of nodes."""
        w = self.w
        nc = w.ncomp
        nx, ny = w.ne[0] + 1, w.ne[1] + 1
        full = w.free_index()
        def ijk(nodes):
            return np.stack([nodes % nx, (nodes // nx) % ny, nodes // (nx * ny)], axis=1)
        weights = []
        for Ib, I in zip(self.Ibar, self.I):
            nodes_I = full[I] // nc
            nodes_bd = np.setdiff1d(full[Ib] // nc, nodes_I)
            wj = np.ones(len(I))
            if len(nodes_bd):
                P, S = ijk(nodes_I), ijk(nodes_bd)
                for s0 in range(0, len(P), 2048):
                    d = np.abs(P[s0:s0 + 2048, None, :] - S[None, :, :]).max(axis=2)
                    wj[s0:s0 + 2048] = d.min(axis=1)
            weights.append(wj)
        total = np.zeros(w.n_free)
        for I, wj in zip(self.I, weights):
            total[I] += wj
        X = []
        for Ib, I, wj in zip(self.Ibar, self.I, weights):
            x = np.zeros(len(Ib))
            x[np.searchsorted(Ib, I)] = wj / total[I]
            X.append(x)
        return X

    def _free_dofs(self, nodes: np.ndarray) -> np.ndarray:
        nc = self.w.ncomp
        full = (nodes[:, None] * nc + np.arange(nc)[None, :]).ravel()
        f = self.free_of_full[full]
        return np.sort(f[f >= 0])

    @property
    def n_sub(self) -> int:
        return len(self.E)

    def pou_sum(self, v: np.ndarray) -> np.ndarray:
        """sum_j R_j^T Xi_j (v restricted to Omega_j)  (Definition of the PoU)."""
        out = np.zeros_like(v)
        for Ib, x in zip(self.Ibar, self.X):
            out[Ib] += x * v[Ib]
        return out
