"""Pins of the oracle's reference adjoint (no GPU).

The adjoint (oracle/oracle_adjoint.c) is checked against central finite
differences of the oracle's own forward objective -- a different code path
(the forward update and wall-shear-stress sum), as the protocol of the
differentiation form asks:
  * every per-step inlet amplitude derivative of a short window;
  * directional derivatives in random porosity directions;
  * the largest single-site porosity derivatives.
Objective: J = sum over t in the window of the summed wall shear stress.
"""
import numpy as np
import pytest

from paper_2202_11770_amd import geometry as G


def _case(orc, nsteps=60, seed=4):
    g = G.tortuous(radius=4.0, length=32, amplitude=4.0, period=32.0)
    rng = np.random.default_rng(seed)
    s = np.arange(nsteps)
    a = rng.uniform(-1, 1, 4) * 0.002 / np.arange(1, 5)
    b = rng.uniform(-1, 1, 4) * 0.002 / np.arange(1, 5)
    A = 0.01 + sum(a[k] * np.cos(2 * np.pi * (k + 1) * s / nsteps) + b[k] * np.sin(2 * np.pi * (k + 1) * s / nsteps)
                   for k in range(4))
    tables = [A if io.kind == G.VELOCITY else np.array([1.0]) for io in g.iolets]
    phi = np.zeros(g.n)
    ws = g.wall_sites()
    phi[ws] = np.random.default_rng(40).uniform(0, 1, ws.size)
    return g, tables, phi, ws


@pytest.fixture(scope="module")
def adj(orc):
    nsteps, w0, w1, tau = 60, 30, 60, 0.8
    g, tables, phi, ws = _case(orc, nsteps)
    P = orc.Problem(g, tau, tables=tables, phi=phi)
    f0 = P.init()
    J, dA, dphi = P.adjoint(f0, 0, nsteps, w0, w1)
    return dict(g=g, tables=tables, phi=phi, ws=ws, P=P, f0=f0, J=J, dA=dA, dphi=dphi, nsteps=nsteps, w=(w0, w1),
                tau=tau)


def _J(orc, d, tables=None, phi=None):
    P = orc.Problem(d["g"], d["tau"], tables=tables if tables is not None else d["tables"],
                    phi=phi if phi is not None else d["phi"])
    return P.objective(d["f0"], 0, d["nsteps"], *d["w"])


def test_objective_matches_forward(orc, adj):
    assert adj["J"] > 0
    assert abs(_J(orc, adj) - adj["J"]) <= 1e-14 * adj["J"]


def test_inlet_amplitude_gradient_fd(orc, adj):
    d = adj
    k = [i for i, io in enumerate(d["g"].iolets) if io.kind == G.VELOCITY][0]
    h = 1e-7
    steps = list(range(0, d["nsteps"], 3))
    fd = []
    for s in steps:
        tp = [t.copy() for t in d["tables"]]
        tm = [t.copy() for t in d["tables"]]
        tp[k][s] += h
        tm[k][s] -= h
        fd.append((_J(orc, d, tables=tp) - _J(orc, d, tables=tm)) / (2 * h))
    fd = np.array(fd)
    ad = d["dA"][k, steps]
    # steps after the window's end cannot influence J
    assert np.all(d["dA"][k, d["w"][1]:] == 0.0)
    err = np.linalg.norm(ad - fd) / np.linalg.norm(fd)
    print("amplitude group rel err", err)
    assert err <= 1e-6
    # pressure iolets get no amplitude derivative
    for kk, io in enumerate(d["g"].iolets):
        if io.kind == G.PRESSURE:
            assert np.all(d["dA"][kk] == 0.0)


def test_porosity_gradient_fd(orc, adj):
    d = adj
    h = 1e-6
    rng = np.random.default_rng(3)
    errs = []
    for _ in range(3):
        v = np.zeros(d["g"].n)
        v[d["ws"]] = rng.uniform(-1, 1, d["ws"].size)
        v /= np.abs(v).max()
        fd = (_J(orc, d, phi=d["phi"] + h * v) - _J(orc, d, phi=d["phi"] - h * v)) / (2 * h)
        ad = float(d["dphi"] @ v)
        errs.append(abs(ad - fd) / abs(fd))
    print("porosity directional rel errs", errs)
    assert max(errs) <= 1e-6
    # sites without wall links have no porosity derivative
    nonwall = np.setdiff1d(np.arange(d["g"].n), d["ws"])
    assert np.all(d["dphi"][nonwall] == 0.0)


def test_porosity_largest_components_fd(orc, adj):
    d = adj
    h = 1e-6
    top = np.argsort(-np.abs(d["dphi"]))[:4]
    fd = []
    for x in top:
        v = np.zeros(d["g"].n)
        v[x] = 1.0
        fd.append((_J(orc, d, phi=d["phi"] + h * v) - _J(orc, d, phi=d["phi"] - h * v)) / (2 * h))
    fd = np.array(fd)
    err = np.linalg.norm(d["dphi"][top] - fd) / np.linalg.norm(fd)
    print("porosity top-4 rel err", err)
    assert err <= 1e-6
