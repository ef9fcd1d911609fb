"""CPU checks of the serving workload generator: catalogue sizes, subdomain
sizes and the layout of patch tractions (interface conventions only)."""
import numpy as np

from workloads import generate as gen


def test_c4_catalogue_sizes():
    cat = gen.config_c4_catalogue()
    assert len(cat) == 16
    targets = [0.2e6] * 4 + [0.5e6] * 4 + [1.0e6] * 4 + [2.0e6] * 4
    for w, S in zip(cat, targets):
        assert abs(w.n_free - S) <= 0.06 * S, (w.name, w.n_free)
        n_ply = (w.ne[2] + 1) // 4
        assert 8 <= n_ply <= 24 and w.ne[2] == 4 * n_ply - 1
        assert 3500 <= w.n_free / w.n_sub <= 6500, w.name
        assert w.body is None and w.overlap == 1 and w.nev == 12
        assert np.all(w.dirichlet.reshape(-1, 3)[:: w.nn[0]] == 1)   # clamped at x = 0


def test_patch_tractions_layout():
    w = gen.small_case("laminate", seed=3, nxy=(10, 6), n_ply=2)
    rng = np.random.default_rng(0)
    t = gen.patch_tractions(w, 4, rng).reshape(4, w.ne[1], w.ne[0], 3)
    for r in range(4):
        nz = np.argwhere(np.any(t[r] != 0, axis=-1))
        assert len(nz) > 0
        # one uniform traction on an axis-aligned rectangle of faces
        (y0, x0), (y1, x1) = nz.min(0), nz.max(0)
        assert len(nz) == (y1 - y0 + 1) * (x1 - x0 + 1)
        vals = t[r][nz[:, 0], nz[:, 1]]
        assert np.all(vals == vals[0])


def test_c4_requests_stream():
    rq = gen.c4_requests(16, n_req=1000)
    t = np.array([r["t"] for r in rq])
    assert np.all(np.diff(t) > 0)
    assert 40.0 < t[-1] < 60.0                       # mean 20 per second
    ks = np.array([r["k"] for r in rq])
    assert ks.min() == 1 and ks.max() == 16
    assert set(r["op"] for r in rq) == set(range(16))
