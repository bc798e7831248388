"""Pins of the oracle's reference adjoint (no GPU).

The adjoint (oracle/oracle_adjoint.c) is checked against central finite
differences of the oracle's own forward objective -- a different code path
(the forward update, the wall-shear-stress sum, the per-iolet outflow), as
the protocol of the differentiation form asks:
  * per-step inlet amplitude derivatives of a short window;
  * per-step outlet ghost-density derivatives;
  * directional derivatives in random porosity directions;
  * the largest single-site porosity derivatives.
Objectives: J = sum over t in the window of the summed wall shear stress
("wss"), or of the outlet's outflow during the update t-1 -> t ("flux").
The outflow itself is pinned by mass conservation and by the Ladd inflow
of a pipe.
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
    # per-step outlet densities, so that each step's value can be perturbed
    R = 1.0 + 0.001 * np.sin(2 * np.pi * s / nsteps)
    tables = [A if io.kind == G.VELOCITY else R.copy() for io in g.iolets]
    phi = np.zeros(g.n)
    ws = g.wall_sites()
    phi[ws] = np.random.default_rng(40).uniform(0, 1, ws.size)
    return g, tables, phi, ws


def _weights(g, objective):
    """None for the WSS objective; for the flux objective the outlet's
    outflow (weight 1 on pressure iolets, 0 on the inlet)."""
    if objective == "wss":
        return None
    return np.array([1.0 if io.kind == G.PRESSURE else 0.0 for io in g.iolets])


@pytest.fixture(scope="module", params=["wss", "flux"])
def adj(orc, request):
    nsteps, w0, w1, tau = 60, 30, 60, 0.8
    g, tables, phi, ws = _case(orc, nsteps)
    P = orc.Problem(g, tau, tables=tables, phi=phi)
    f0 = P.init()
    wts = _weights(g, request.param)
    J, dA, dphi = P.adjoint(f0, 0, nsteps, w0, w1, weights=wts)
    return dict(g=g, tables=tables, phi=phi, ws=ws, P=P, f0=f0, J=J, dA=dA, dphi=dphi, nsteps=nsteps, w=(w0, w1),
                tau=tau, weights=wts, objective=request.param)


def _J(orc, d, tables=None, phi=None):
    P = orc.Problem(d["g"], d["tau"], tables=tables if tables is not None else d["tables"],
                    phi=phi if phi is not None else d["phi"])
    return P.objective(d["f0"], 0, d["nsteps"], *d["w"], weights=d["weights"])


def test_objective_matches_forward(orc, adj):
    assert adj["J"] != 0
    assert abs(_J(orc, adj) - adj["J"]) <= 1e-14 * abs(adj["J"])


def _table_fd(orc, d, kind, h):
    k = [i for i, io in enumerate(d["g"].iolets) if io.kind == kind][0]
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
    return np.linalg.norm(ad - fd) / np.linalg.norm(fd)


def test_inlet_amplitude_gradient_fd(orc, adj):
    err = _table_fd(orc, adj, G.VELOCITY, 1e-7)
    print(adj["objective"], "amplitude group rel err", err)
    assert err <= 1e-6


def test_outlet_density_gradient_fd(orc, adj):
    err = _table_fd(orc, adj, G.PRESSURE, 1e-6)
    print(adj["objective"], "ghost density group rel err", err)
    assert err <= 1e-6


def _h_phi(d):
    """Porosity FD step.  The outflow objective is a sum of differences of
    O(w_i) populations, so its rounding noise is larger than the WSS sum's:
    a step study on this case gives FD-vs-adjoint errors of 6e-10..3e-9 at
    h = 1e-4, 3e-8..6e-8 at 1e-5, 1e-7..2e-6 at 1e-6 (rounding-dominated)."""
    return 1e-6 if d["objective"] == "wss" else 1e-4


def test_porosity_gradient_fd(orc, adj):
    d = adj
    h = _h_phi(d)
    rng = np.random.default_rng(3)
    errs = []
    for _ in range(3):
        v = np.zeros(d["g"].n)
        v[d["ws"]] = rng.uniform(-1, 1, d["ws"].size)
        v /= np.abs(v).max()
        fd = (_J(orc, d, phi=d["phi"] + h * v) - _J(orc, d, phi=d["phi"] - h * v)) / (2 * h)
        ad = float(d["dphi"] @ v)
        errs.append(abs(ad - fd) / abs(fd))
    print(d["objective"], "porosity directional rel errs", errs)
    assert max(errs) <= 1e-6
    # sites without wall links have no porosity derivative
    nonwall = np.setdiff1d(np.arange(d["g"].n), d["ws"])
    assert np.all(d["dphi"][nonwall] == 0.0)


def test_porosity_largest_components_fd(orc, adj):
    d = adj
    h = _h_phi(d)
    top = np.argsort(-np.abs(d["dphi"]))[:4]
    fd = []
    for x in top:
        v = np.zeros(d["g"].n)
        v[x] = 1.0
        fd.append((_J(orc, d, phi=d["phi"] + h * v) - _J(orc, d, phi=d["phi"] - h * v)) / (2 * h))
    fd = np.array(fd)
    err = np.linalg.norm(d["dphi"][top] - fd) / np.linalg.norm(fd)
    print(d["objective"], "porosity top-4 rel err", err)
    assert err <= 1e-6


def test_outflow_is_mass_loss(orc):
    """With weight 1 on every iolet and no porosity, the summed outflow of the
    updates in (t0, t1] is the mass lost between t0 and t1: the collision and
    bounce-back conserve mass (checked through the plain sum of f)."""
    nsteps = 40
    g, tables, _, _ = _case(orc, nsteps)
    P = orc.Problem(g, 0.8, tables=tables)
    f = P.init()
    P.run(f, 0, 10)  # away from rest
    m0 = P.mass(f)
    Qsum = 0.0
    for t in range(10, 30):
        Qsum += P.iolet_flux(f, t).sum()
        P.run(f, t, 1)
    loss = m0 - P.mass(f)
    print("outflow", Qsum, "mass loss", loss)
    assert abs(Qsum) > 1e-3
    assert abs(Qsum - loss) <= 1e-12 * P.mass(f)


def test_ladd_inflow_of_pipe(orc):
    """The pipe's parabolic Ladd inlet (u_max 0.01, radius 8) lets in about
    rho0 u_max pi R^2 / 2 per step (the sum over inlet links of
    6 w_i rho0 |c_i.n| A W(m) is A W per cross-section site)."""
    g = G.cylinder()
    P = orc.Problem(g, 0.8)
    f = P.init()
    Q = P.iolet_flux(f, 0)
    k_in = [k for k, io in enumerate(g.iolets) if io.kind == G.VELOCITY][0]
    expect = -1.0 * 0.01 * np.pi * 8.0 ** 2 / 2
    print("inlet outflow", Q[k_in], "expected", expect)
    assert abs(Q[k_in] / expect - 1) < 0.05
