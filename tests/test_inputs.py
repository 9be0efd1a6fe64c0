"""The seeded input generators (paper_2107_03632_amd.nodes): the recipes the
workloads are built from, checked on the CPU.  They hold no method
arithmetic, only node sets."""

import numpy as np

from paper_2107_03632_amd import nodes


def test_jittered_cube_recipe():
    q = 9
    x, y, z = nodes.jittered_cube(q, seed=6)
    x2, y2, z2 = nodes.jittered_cube(q, seed=6)
    assert x.shape == (q ** 3,) and np.array_equal(x, x2) and np.array_equal(z, z2)
    h = 1.0 / q
    g = (np.arange(q) + 0.5) * h
    # lattice order, x fastest, each coordinate within 0.25 h of its site
    ix = np.tile(g, q * q)
    iy = np.tile(np.repeat(g, q), q)
    iz = np.repeat(g, q * q)
    for a, c in ((x, ix), (y, iy), (z, iz)):
        assert np.abs(a - c).max() <= 0.25 * h + 1e-15
        assert np.abs(a - c).max() > 0.2 * h   # the jitter is there
    assert not np.array_equal(x, nodes.jittered_cube(q, seed=7)[0])


def test_unit_disk_recipe():
    ns = nodes.unit_disk(20_000, 300, seed=2)
    r = np.hypot(ns.x, ns.y)
    bnd = ns.is_boundary == 1
    assert bnd.sum() == 300
    assert np.allclose(r[bnd], 1.0)
    assert r[~bnd].max() < 1.0
    ns2 = nodes.unit_disk(20_000, 300, seed=2)
    assert np.array_equal(ns.x, ns2.x) and np.array_equal(ns.y, ns2.y)
    # minimum spacing of the jittered lattice stays >= h/2 (Poisson-disk-like)
    from scipy.spatial import cKDTree
    pts = np.stack([ns.x[~bnd], ns.y[~bnd]], 1)
    d, _ = cKDTree(pts).query(pts, k=2)
    assert d[:, 1].min() >= 0.5 * ns.h * (1 - 1e-12)
