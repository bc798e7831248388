"""Windkessel outlets on the GPU (hlb_set_windkessel) against the oracle's
Problem.run_windkessel: macros and the outlet states after n steps."""
import numpy as np
import pytest

import oracle
from paper_2202_11770_amd import geometry as G
from paper_2202_11770_amd import hlb
from _parity import check_bars, errors, fmt

pytestmark = pytest.mark.gpu


def _case(name):
    if name == "pipe":
        g = G.cylinder()
        k = [k for k, io in enumerate(g.iolets) if io.kind == G.PRESSURE][0]
        return g, None, 0.8, 600, {k: (1.0, 0.001, 2000.0, 0.002, 0.0)}
    g = G.tree(seed=3, generations=3, target_sites=30000)
    s = np.arange(200)
    tables = [0.02 * 0.5 * (1 - np.cos(2 * np.pi * s / 200)) if io.kind == G.VELOCITY else None for io in g.iolets]
    outs = [k for k, io in enumerate(g.iolets) if io.kind == G.PRESSURE]
    # a different model per outlet: resistances, capacitors, one pure resistance
    models = {}
    for j, k in enumerate(outs):
        C = 0.0 if j == 0 else 500.0 * (j + 1)
        models[k] = (1.0, 0.002 * (j + 1), C, 0.004, 0.0005 * j if C > 0 else 0.0)
    return g, tables, 0.6, 300, models


@pytest.mark.parametrize("scheme", ["pull", "push"])
@pytest.mark.parametrize("name", ["pipe", "tree"])
def test_windkessel_matches_oracle(name, scheme):
    g, tables, tau, steps, models = _case(name)
    print(f"case: {name} {g.n} sites, {len(models)} Windkessel outlets, {steps} steps, {scheme}", flush=True)
    P = oracle.Problem(g, tau, tables=tables)
    f = P.init()
    ref_state = P.run_windkessel(f, 0, steps, models)
    ref = P.macros(f)
    sim = hlb.Simulation.create(g, tau, tables=tables, scheme=scheme)
    for k, m in models.items():
        hlb.hlb_set_windkessel(sim.ctx, k, m)
    sim.step(steps)
    rho, u, wss = sim.macros()
    e = errors(rho, u, wss, *ref)
    worst = 0.0
    for k in models:
        got = hlb.hlb_windkessel_state(sim.ctx, k)
        want = ref_state[k]
        worst = max(worst, abs(got[0] - want[0]), abs(got[1] - want[1]) / max(abs(want[1]), 1e-12),
                    abs(got[2] - want[2]) / max(abs(want[2]), 1e-12))
    print(f"{name} {scheme}: {fmt(e)}; worst outlet-state error {worst:.2e}", flush=True)
    sim.close()
    assert e["e_rho"] <= 1e-12 and e["e_u"] <= 1e-12 and e["e_wss"] <= 1e-10
    assert worst <= 1e-11


def test_windkessel_fp32_and_errors():
    g, tables, tau, steps, models = _case("tree")
    P = oracle.Problem(g, tau, tables=tables)
    f = P.init()
    P.run_windkessel(f, 0, steps, models)
    ref = P.macros(f)
    sim = hlb.Simulation.create(g, tau, storage="f32", tables=tables)
    for k, m in models.items():
        hlb.hlb_set_windkessel(sim.ctx, k, m)
    sim.step(steps)
    e = errors(*sim.macros(), *ref)
    print(f"tree f32 Windkessel: {fmt(e)}", flush=True)
    check_bars(e, dict(e_rho=2e-7, e_u=5e-6, e_wss=1e-5), "Windkessel f32")
    k_vel = [k for k, io in enumerate(g.iolets) if io.kind == G.VELOCITY][0]
    k_out = next(iter(models))
    with pytest.raises(hlb.HLBError, match="not a pressure iolet"):
        hlb.hlb_set_windkessel(sim.ctx, k_vel, (1.0, 0.0, 0.0, 0.0, 0.0))
    with pytest.raises(hlb.HLBError, match="R2 C"):
        hlb.hlb_set_windkessel(sim.ctx, k_out, (1.0, 0.0, 10.0, 0.01, 0.0))
    # a table replaces the model
    hlb.hlb_set_iolet_table(sim.ctx, k_out, [1.0])
    with pytest.raises(hlb.HLBError, match="not a Windkessel"):
        hlb.hlb_windkessel_state(sim.ctx, k_out)
    sim.close()
    # the adjoint carries the model (parity: tests/test_gpu_adjoint_windkessel.py)
    # and leaves the model's state as it found it
    adj = hlb.Simulation.create(g, tau, tables=tables, adjoint=True)
    hlb.hlb_set_windkessel(adj.ctx, k_out, (1.0, 0.001, 0.0, 0.001, 0.0))
    adj.step(5)
    before = hlb.hlb_windkessel_state(adj.ctx, k_out)
    J, dA, dphi, fw = hlb.hlb_adjoint_run(adj.ctx, 10, 5, 15, 2)
    assert np.isfinite(J) and J > 0 and np.all(np.isfinite(dA))
    assert hlb.hlb_windkessel_state(adj.ctx, k_out) == before
    adj.close()
