"""Pins of the oracle's single-site algebra (no GPU).

Checks the oracle against facts fixed outside its own code:
* the velocity set and weights printed in the paper (Sec. 2.2), from a
  golden text fixture;
* lattice isotropy (the moments that make the scheme recover Navier-Stokes);
* the moment identities that the equilibrium of eq. (4) must satisfy -- the
  second moment rho/3 delta + rho u u fails for the printed form without the
  1/2 factors, so it pins that reading;
* conservation of rho and rho u by the collision of eq. (3a) and the linear
  relaxation f' - f^eq = (1 - 1/tau)(f - f^eq), computed in exact rational
  arithmetic from the oracle's own outputs.
"""
import itertools
import os
from fractions import Fraction

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden", "d3q19_lattice.txt")


def _golden():
    groups = {}
    cs2 = None
    for line in open(GOLD):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        parts = line.split()
        if parts[0] == "cs2":
            cs2 = Fraction(parts[1])
            continue
        w = Fraction(parts[1])
        vecs = [tuple(int(v) for v in p.strip("()").split(",")) for p in parts[2:]]
        groups[parts[0]] = (w, vecs)
    return groups, cs2


def test_lattice_matches_paper(orc):
    c, w, opp = orc.lattice()
    groups, cs2 = _golden()
    assert cs2 == Fraction(1, 3)
    # same set of 19 vectors, with the printed weight for each
    want = {}
    for name, (wt, vecs) in groups.items():
        for v in vecs:
            want[v] = wt
    assert len(want) == 19
    got = {tuple(int(a) for a in c[i]): w[i] for i in range(19)}
    assert set(got) == set(want)
    for v, wt in want.items():
        assert got[v] == pytest.approx(float(wt), rel=0, abs=1e-17)
    # the paper's grouping: i = 0 rest, 1-6 axis, 7-18 diagonals
    assert tuple(c[0]) == (0, 0, 0)
    assert all(tuple(c[i]) in groups["axis"][1] for i in range(1, 7))
    assert all(tuple(c[i]) in groups["diag"][1] for i in range(7, 19))
    # opposite table
    for i in range(19):
        assert tuple(c[opp[i]]) == tuple(-c[i])


def test_lattice_isotropy(orc):
    c, w, _ = orc.lattice()
    wf = [Fraction(1, 3)] + [Fraction(1, 18)] * 6 + [Fraction(1, 36)] * 12
    for i in range(19):
        assert float(wf[i]) == w[i]
    assert sum(wf) == 1
    for a in range(3):
        assert sum(wf[i] * c[i][a] for i in range(19)) == 0
        for b in range(3):
            m2 = sum(wf[i] * c[i][a] * c[i][b] for i in range(19))
            assert m2 == (Fraction(1, 3) if a == b else 0)
    for a, b, cc, d in itertools.product(range(3), repeat=4):
        m4 = sum(wf[i] * c[i][a] * c[i][b] * c[i][cc] * c[i][d] for i in range(19))
        want = Fraction(int(a == b) * int(cc == d) + int(a == cc) * int(b == d) + int(a == d) * int(b == cc), 9)
        assert m4 == want


def _rand_state(rng):
    rho = 1.0 + rng.uniform(-0.05, 0.05)
    u = rng.uniform(-0.05, 0.05, 3)
    return rho, u


@pytest.mark.parametrize("seed", range(20))
def test_equilibrium_moments(orc, seed):
    rng = np.random.default_rng(seed)
    c, _, _ = orc.lattice()
    rho, u = _rand_state(rng)
    feq = orc.equilibrium(rho, u)
    assert feq.sum() == pytest.approx(rho, rel=1e-15)
    assert np.allclose(feq @ c, rho * u, rtol=0, atol=1e-16)
    P = np.einsum("i,ia,ib->ab", feq, c, c)
    want = rho * np.eye(3) / 3.0 + rho * np.outer(u, u)
    assert np.allclose(P, want, rtol=0, atol=2e-16)
    # the printed form (no 1/2 factors) would give rho/3 + 2 rho u u - rho |u|^2 ...: far from this
    assert np.abs(P - want).max() < 1e-3 * np.abs(np.outer(u, u)).max()


@pytest.mark.parametrize("seed", range(20))
def test_collision_exact(orc, seed):
    """Conservation and linear relaxation, checked in exact rationals."""
    rng = np.random.default_rng(100 + seed)
    c, _, _ = orc.lattice()
    tau = 0.8
    rho, u = _rand_state(rng)
    f = orc.equilibrium(rho, u) + rng.uniform(-1e-3, 1e-3, 19)
    fp = orc.collide(f, tau)
    F = [Fraction(v) for v in f]
    FP = [Fraction(v) for v in fp]
    # mass and momentum conserved up to the rounding of 19 terms
    dm = sum(FP) - sum(F)
    assert abs(float(dm)) <= 19 * 2.0 ** -53 * 4
    for a in range(3):
        dj = sum((FP[i] - F[i]) * int(c[i][a]) for i in range(19))
        assert abs(float(dj)) <= 19 * 2.0 ** -53 * 4
    # f' - feq = (1 - 1/tau)(f - feq), feq from the exact moments of f
    r, v = orc.moments(f)
    feq = orc.equilibrium(r, v)
    for i in range(19):
        lhs = FP[i] - Fraction(feq[i])
        rhs = (1 - 1 / Fraction(tau)) * (F[i] - Fraction(feq[i]))
        assert abs(float(lhs - rhs)) <= 4 * 2.0 ** -53


def test_equilibrium_rest_and_special_cases(orc):
    _, w, _ = orc.lattice()
    assert np.array_equal(orc.equilibrium(1.0, [0, 0, 0]), w)
    assert np.array_equal(orc.equilibrium(2.0, [0, 0, 0]), 2 * w)
    # collision leaves an equilibrium unchanged (tau = 1 projects onto it)
    f = orc.equilibrium(1.01, [0.01, -0.02, 0.005])
    assert np.allclose(orc.collide(f, 0.6), f, rtol=0, atol=2e-16)
    g = f + np.linspace(-1e-4, 1e-4, 19)
    r, v = orc.moments(g)
    assert np.allclose(orc.collide(g, 1.0), orc.equilibrium(r, v), rtol=0, atol=2e-16)
