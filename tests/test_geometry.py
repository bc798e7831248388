"""Input generators: neighbour-table symmetry, site classes, sizes (no GPU)."""
import math

import numpy as np
import pytest

from paper_2202_11770_amd import geometry as G


def _check_table(g):
    n = g.n
    nbr = g.nbr
    assert nbr.shape == (n, 19)
    assert np.array_equal(nbr[:, 0], np.arange(n))
    # symmetric: nbr[x][i] = y  =>  nbr[y][opp i] = x
    for i in range(1, 19):
        y = nbr[:, i]
        m = y >= 0
        assert np.array_equal(nbr[y[m], G.OPP[i]], np.nonzero(m)[0])
    # site types agree with the link codes
    wall = (nbr == -1).any(axis=1)
    io = nbr <= -2
    has_io = io.any(axis=1)
    t = g.types
    assert np.all((t == G.SITE_BULK) == (~wall & ~has_io))
    assert np.all((t == G.SITE_WALL) == (wall & ~has_io))
    assert np.all(np.isin(t[has_io], [2, 3, 4, 5]))
    assert np.all(wall[np.isin(t, [4, 5])])


def test_cylinder_classes():
    g = G.cylinder()
    assert g.n == 13312  # 208 sites per slice x 64 slices
    assert np.bincount(g.types, minlength=6).tolist() == [9176, 3720, 148, 148, 60, 60]
    _check_table(g)
    # coordinates of fluid neighbours differ by c_i
    for i in range(1, 19):
        y = g.nbr[:, i]
        m = y >= 0
        assert np.array_equal(g.coords[y[m]] - g.coords[m], np.broadcast_to(G.C[i], (m.sum(), 3)))
    assert abs(g.n / (math.pi * 64 * 64) - 1) < 0.05


@pytest.mark.parametrize("maker", ["duct", "sealed", "periodic", "couette", "tortuous", "tree"])
def test_tables(maker):
    g = {"duct": lambda: G.duct(8, 12, 20), "sealed": lambda: G.sealed_box(6, 7, 8),
         "periodic": lambda: G.periodic_box(4, 5, 6), "couette": lambda: G.couette_column(5),
         "tortuous": lambda: G.tortuous(radius=6, length=64, amplitude=6, period=64),
         "tree": lambda: G.tree(seed=3, generations=3, target_sites=30000)}[maker]()
    _check_table(g)


def test_tree_reproducible_and_scaled():
    a = G.tree(seed=5, generations=4, target_sites=50000)
    b = G.tree(seed=5, generations=4, target_sites=50000)
    assert np.array_equal(a.nbr, b.nbr) and np.array_equal(a.coords, b.coords)
    assert abs(a.n - 50000) <= 0.01 * 50000
    assert len(a.iolets) == 1 + 2 ** 4
    assert sum(io.role == G.INLET for io in a.iolets) == 1
    c = G.tree(seed=6, generations=4, target_sites=50000)
    assert not np.array_equal(a.coords[:100], c.coords[:100]) or a.n != c.n


def test_permute_roundtrip():
    g = G.cylinder()
    perm = np.random.default_rng(0).permutation(g.n)
    gp = G.permute(g, perm)
    _check_table(gp)
    assert np.array_equal(gp.coords, g.coords[perm])
    inv = np.empty_like(perm)
    inv[perm] = np.arange(g.n)
    back = G.permute(gp, inv)
    assert np.array_equal(back.nbr, g.nbr)
