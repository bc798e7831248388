"""Pins of the oracle's tangent-linear model and, through it, of the
reference adjoint (no GPU).

  * The tangent-linear model (oracle/oracle_tangent.c, forward mode) against
    central finite differences of the oracle's forward objective in random
    directions of the initial state, the per-step table values and the
    porosity: pins the model itself.
  * The dot-product identity  dJ[v] = <grad J, v>  between the tangent-linear
    model and the reference adjoint (oracle/oracle_adjoint.c, reverse mode),
    for random directions v of all inputs at once.  The two codes are written
    independently (one propagates perturbations through the forward update,
    the other transposes per-site Jacobians), so agreement to rounding pins
    every index, opposite direction and sign of the transposition -- a far
    tighter bar than the finite-difference checks.
Both objectives (summed wall shear stress, weighted iolet outflow), with
porous walls, a Ladd inlet and a ghost-density outlet.
"""
import numpy as np
import pytest

from paper_2202_11770_amd import geometry as G

NSTEPS, W0, W1, TAU = 40, 20, 40, 0.8


def _case(seed=4):
    g = G.tortuous(radius=4.0, length=32, amplitude=4.0, period=32.0)
    s = np.arange(NSTEPS)
    rng = np.random.default_rng(seed)
    A = 0.01 + 0.002 * np.sin(2 * np.pi * s / NSTEPS + rng.uniform(0, 2 * np.pi))
    R = 1.0 + 0.001 * np.sin(2 * np.pi * s / NSTEPS)
    tables = [A.copy() if io.kind == G.VELOCITY else R.copy() for io in g.iolets]
    phi = np.zeros(g.n)
    ws = g.wall_sites()
    phi[ws] = np.random.default_rng(40).uniform(0, 1, ws.size)
    return g, tables, phi, ws


def _weights(g, objective):
    if objective == "wss":
        return None
    # inlet and outlet both weighted, with different weights
    return np.array([0.5 if io.kind == G.VELOCITY else 1.0 for io in g.iolets])


@pytest.fixture(scope="module", params=["wss", "flux"])
def case(orc, request):
    g, tables, phi, ws = _case()
    P = orc.Problem(g, TAU, tables=tables, phi=phi)
    # a non-equilibrium, moving initial state
    rng = np.random.default_rng(11)
    rho = 1.0 + 0.002 * rng.standard_normal(g.n)
    u = 0.005 * rng.standard_normal((g.n, 3))
    f0 = P.init(rho, u)
    return dict(g=g, tables=tables, phi=phi, ws=ws, P=P, f0=f0, weights=_weights(g, request.param),
                objective=request.param)


def _direction(d, seed, scale_f=1e-3, scale_tab=1e-3, scale_phi=0.1):
    rng = np.random.default_rng(seed)
    n, n_io = d["g"].n, len(d["g"].iolets)
    df0 = scale_f * rng.standard_normal((n, 19)) / 19
    dtab = scale_tab * rng.standard_normal((n_io, NSTEPS))
    dphi = np.zeros(n)
    dphi[d["ws"]] = scale_phi * rng.uniform(-1, 1, d["ws"].size)
    return df0, dtab, dphi


def _J(orc, d, f0, tables, phi):
    P = orc.Problem(d["g"], TAU, tables=tables, phi=phi)
    return P.objective(f0, 0, NSTEPS, W0, W1, weights=d["weights"])


def test_tangent_vs_central_differences(orc, case):
    d = case
    # h small enough for the O(h^2) truncation to sit far below 1e-6 and large
    # enough for rounding (the flux objective is a difference of O(w_i)
    # populations) to stay below it
    for part, h in (("state", 1e-4), ("tables", 1e-4), ("porosity", 1e-3), ("all", 1e-4)):
        df0, dtab, dphi = _direction(d, seed={"state": 21, "tables": 22, "porosity": 23, "all": 24}[part])
        if part != "all":
            df0 = df0 if part == "state" else None
            dtab = dtab if part == "tables" else None
            dphi = dphi if part == "porosity" else None
        tl = d["P"].tangent(d["f0"], 0, NSTEPS, W0, W1, weights=d["weights"], df0=df0, dtab=dtab, dphi=dphi)

        def shifted(sign):
            f0 = d["f0"] + sign * h * (df0 if df0 is not None else 0.0)
            tabs = [t + sign * h * (dtab[k] if dtab is not None else 0.0) for k, t in enumerate(d["tables"])]
            phi = d["phi"] + sign * h * (dphi if dphi is not None else 0.0)
            return _J(orc, d, f0, tabs, phi)

        fd = (shifted(+1) - shifted(-1)) / (2 * h)
        err = abs(tl - fd) / abs(fd)
        print(f"{d['objective']} {part}: tangent {tl:.12e} FD {fd:.12e} rel {err:.2e}")
        assert fd != 0.0
        assert err <= 1e-6


def test_dot_product_identity(orc, case):
    """dJ[v] from the tangent-linear model equals <grad J, v> from the adjoint."""
    d = case
    J, dA, dphi_g, df0_g = d["P"].adjoint(d["f0"], 0, NSTEPS, W0, W1, weights=d["weights"], state_grad=True)
    for seed in (1, 2, 3):
        df0, dtab, dphi = _direction(d, seed)
        tl = d["P"].tangent(d["f0"], 0, NSTEPS, W0, W1, weights=d["weights"], df0=df0, dtab=dtab, dphi=dphi)
        terms = np.concatenate([(df0_g * df0).ravel(), (dA * dtab).ravel(), dphi_g * dphi])
        dot = float(np.sum(terms))
        scale = float(np.sum(np.abs(terms)))
        err = abs(tl - dot) / scale
        print(f"{d['objective']} seed {seed}: tangent {tl:.15e} adjoint {dot:.15e} rel (to sum |terms|) {err:.2e}")
        assert err <= 1e-12
    # each input group on its own, so that a group with a small share of the
    # total cannot hide a mismatch
    df0, dtab, dphi = _direction(d, 7)
    for part, kw, terms in (("state", dict(df0=df0), df0_g * df0), ("tables", dict(dtab=dtab), dA * dtab),
                            ("porosity", dict(dphi=dphi), dphi_g * dphi)):
        tl = d["P"].tangent(d["f0"], 0, NSTEPS, W0, W1, weights=d["weights"], **kw)
        dot = float(np.sum(terms))
        err = abs(tl - dot) / float(np.sum(np.abs(terms)))
        print(f"{d['objective']} {part} only: rel {err:.2e}")
        assert err <= 1e-12


def test_tangent_is_zero_outside_window_and_linear(orc, case):
    d = case
    df0, dtab, dphi = _direction(d, 5)
    # table perturbations at steps whose effect cannot reach the window
    late = np.zeros_like(dtab)
    late[:, W1:] = dtab[:, W1:]
    assert d["P"].tangent(d["f0"], 0, NSTEPS, W0, W1, weights=d["weights"], dtab=late) == 0.0
    a = d["P"].tangent(d["f0"], 0, NSTEPS, W0, W1, weights=d["weights"], df0=df0)
    b = d["P"].tangent(d["f0"], 0, NSTEPS, W0, W1, weights=d["weights"], df0=-2.0 * df0)
    assert abs(b + 2.0 * a) <= 1e-14 * abs(a)
