"""The push-order step kernel (hlb_options.scheme = HLB_SCHEME_PUSH): the
paper's own order -- collide the site's pre-collision state, scatter the
results -- against the FP64 oracle, against the pull kernel, and through the
state-exchange entry points.
"""
import numpy as np
import pytest

import oracle
from paper_2202_11770_amd import geometry as G
from paper_2202_11770_amd import hlb
from _parity import check_bars, errors, fmt

pytestmark = pytest.mark.gpu


def _tree(steps):
    g = G.tree(seed=3, generations=3, target_sites=30000)
    s = np.arange(200)
    tables = [0.02 * 0.5 * (1 - np.cos(2 * np.pi * s / 200)) if io.kind == G.VELOCITY else
              1.0 + 0.001 * np.sin(2 * np.pi * s / 200) for io in g.iolets]
    return g, tables


def _run(g, tau, steps, storage, scheme, tables=None, phi=None, order="lex"):
    sim = hlb.Simulation.create(g, tau, storage=storage, tables=tables, scheme=scheme, order=order)
    if phi is not None:
        hlb.hlb_set_porosity(sim.ctx, phi)
    sim.step(steps)
    out = sim.macros()
    m, r = hlb.hlb_mass_balance(sim.ctx)
    sim.close()
    return out, m, r


@pytest.mark.parametrize("case", ["cylinder", "tree", "porous_tree"])
def test_push_fp64_matches_oracle_and_pull(case):
    phi = None
    if case == "cylinder":
        g, tau, steps, tables = G.cylinder(), 0.8, 2000, None
    else:
        g, tables = _tree(400)
        tau, steps = 0.6, 400
        if case == "porous_tree":
            phi = np.zeros(g.n)
            ws = g.wall_sites()
            phi[ws] = np.random.default_rng(7).uniform(0, 0.3, ws.size)
            steps = 300
    print(f"case: {case} {g.n} sites, {steps} steps, push vs oracle and pull", flush=True)
    P = oracle.Problem(g, tau, tables=tables, phi=phi)
    f = P.init()
    P.run(f, 0, steps)
    ref = P.macros(f)
    (rho, u, wss), m, r = _run(g, tau, steps, "f64", "push", tables, phi)
    e = errors(rho, u, wss, *ref)
    (rho_p, u_p, wss_p), m_p, _ = _run(g, tau, steps, "f64", "pull", tables, phi)
    d = errors(rho, u, wss, rho_p, u_p, wss_p)
    print(f"push vs oracle: {fmt(e)}; push vs pull: {fmt(d)}; mass residual {r / m:.2e}", flush=True)
    assert e["e_rho"] <= 1e-12 and e["e_u"] <= 1e-12 and (e["e_wss"] is None or e["e_wss"] <= 1e-10)
    assert abs(m - P.mass(f)) / m <= 1e-12 and abs(m - m_p) / m <= 1e-13
    assert abs(r) / m <= steps * 19 * 2.0 ** -53 / tau


def test_push_reduced_precision():
    g, tables = _tree(400)
    tau, steps = 0.6, 400
    P = oracle.Problem(g, tau, tables=tables)
    f = P.init()
    P.run(f, 0, steps)
    ref = P.macros(f)
    res = {}
    for st in ("f32", "f16"):
        (rho, u, wss), m, r = _run(g, tau, steps, st, "push", tables)
        res[st] = errors(rho, u, wss, *ref)
        print(f"push {st}: {fmt(res[st])} mass residual {r / m:.2e}", flush=True)
    check_bars(res["f32"], dict(e_rho=3e-7, e_u=1e-5, e_wss=2e-5), "push f32")
    check_bars(res["f16"], dict(e_rho=3e-5, e_u=2e-3, e_wss=5e-3), "push f16")


def test_push_state_exchange():
    g, tables = _tree(200)
    tau = 0.6
    sim = hlb.Simulation.create(g, tau, tables=tables, scheme="push")
    assert sim.info()["scheme"] == hlb.HLB_SCHEME_PUSH
    sim.step(37)
    f = sim.state()
    P = oracle.Problem(g, tau, tables=tables)
    fo = P.init()
    P.run(fo, 0, 37)
    assert np.abs(f - fo).max() <= 1e-12
    # set_state then step == stepping on: both continue from the same f(37)
    ref = hlb.Simulation.create(g, tau, tables=tables, scheme="push")
    ref.step(60)
    hlb.hlb_set_state(sim.ctx, f, 37)
    sim.step(23)
    a, b = sim.state(), ref.state()
    assert np.abs(a - b).max() <= 1e-15
    # snapshot and bit-exact state save/load
    hlb.hlb_snapshot_alloc(sim.ctx, 1)
    hlb.hlb_snapshot_save(sim.ctx, 0)
    sim.step(5)
    x = sim.state()
    hlb.hlb_snapshot_restore(sim.ctx, 0)
    sim.step(5)
    assert np.array_equal(sim.state(), x)
    buf = hlb.hlb_state_save(sim.ctx)
    sim.step(3)
    y = sim.state()
    hlb.hlb_state_load(sim.ctx, buf)
    sim.step(3)
    assert np.array_equal(sim.state(), y)
    # a pull context refuses a push state
    pull = hlb.Simulation.create(g, tau, tables=tables)
    with pytest.raises(hlb.HLBError, match="does not match"):
        hlb.hlb_state_load(pull.ctx, buf)
    for s_ in (sim, ref, pull):
        s_.close()


def test_push_rejects_adjoint():
    g = G.cylinder()
    with pytest.raises(hlb.HLBError, match="pull scheme"):
        hlb.Simulation.create(g, 0.8, scheme="push", adjoint=True)
