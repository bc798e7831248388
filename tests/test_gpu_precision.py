"""Precision form: populations stored as FP32 / FP16 deviations f - w rho0,
collided in FP32, against the FP64 oracle.

Targets: FP32 e_rho, e_u, e_wss <= 1e-5 (relative metrics of
tests/_parity.py); FP16 errors are stated.  Each case's bars sit about 3x
above the errors measured on MI355X.
"""
import numpy as np
import pytest

import oracle
from paper_2202_11770_amd import geometry as G
from paper_2202_11770_amd import hlb
from _parity import check_bars, errors, fmt

pytestmark = pytest.mark.gpu


def _run(g, tau, steps, storage, tables=None):
    sim = hlb.Simulation.create(g, tau, storage=storage, tables=tables)
    sim.step(steps)
    out = sim.macros()
    m, r = hlb.hlb_mass_balance(sim.ctx)
    sim.close()
    return out, m, r


BARS = {
    "cylinder": {"f32": dict(e_rho=2e-8, e_u=1e-5, e_wss=5e-6), "f16": dict(e_rho=5e-5, e_u=5e-3, e_wss=3e-3)},
    "tree": {"f32": dict(e_rho=3e-7, e_u=1e-5, e_wss=2e-5), "f16": dict(e_rho=3e-5, e_u=2e-3, e_wss=5e-3)},
}


@pytest.mark.parametrize("case", ["cylinder", "tree"])
def test_storage_errors(case):
    if case == "cylinder":
        g, tau, steps, tables = G.cylinder(), 0.8, 2000, None
    else:
        g = G.tree(seed=3, generations=3, target_sites=30000)
        s = np.arange(200)
        tables = [0.02 * 0.5 * (1 - np.cos(2 * np.pi * s / 200)) if io.kind == G.VELOCITY else np.array([1.0])
                  for io in g.iolets]
        tau, steps = 0.6, 400
    P = oracle.Problem(g, tau, tables=tables)
    f = P.init()
    P.run(f, 0, steps)
    ref = P.macros(f)
    res = {}
    for st in ("f64", "f32", "f16"):
        (rho, u, wss), m, r = _run(g, tau, steps, st, tables)
        res[st] = errors(rho, u, wss, *ref)
        print(f"{case} {st}: {fmt(res[st])} mass_residual_rel={r / m:.2e}", flush=True)
    assert res["f64"]["e_rho"] <= 1e-12 and res["f64"]["e_u"] <= 1e-12
    check_bars(res["f32"], BARS[case]["f32"], f"{case} f32")
    check_bars(res["f16"], BARS[case]["f16"], f"{case} f16")
