"""GPU adjoint through Windkessel outlets, against the oracle's reference
adjoint (orc_adj_run_wk), itself pinned by central differences
(tests/test_oracle_windkessel_adjoint.py).

The tortuous vessel's outlet takes its density from a three-element model
(resistor-capacitor-resistor, capacitor without leak, pure resistance); the
sweep recomputes the forward states, and the model's state, from 4
checkpoints, so the checkpoints must carry that state.  Compared: J, the
table-value derivatives (the inlet's amplitudes and the outlet's per-step
density) and the porosity derivatives, for the WSS and the outflow
objectives.  The model's state and the caller's time are left as they were.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2202_11770_amd import geometry as G
from paper_2202_11770_amd import hlb

pytestmark = pytest.mark.gpu

# (rho_ref, R1, C, R2, X0); the same models as the oracle's pins
MODELS = {
    "rcr": (1.0013, 0.004, 400.0, 0.006, 0.0005),
    "rc_no_leak": (1.0009, 0.003, 300.0, 0.0, -0.0003),
    "resistance": (1.0013, 0.005, 0.0, 0.004, 0.0),
}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


def _case(nsteps=60, seed=4):
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
    return g, tables, phi


@pytest.mark.parametrize("objective", ["wss", "flux"])
@pytest.mark.parametrize("model", list(MODELS))
def test_adjoint_through_windkessel_matches_oracle(model, objective):
    nsteps, w0, w1, tau, n_snap = 60, 30, 60, 0.8, 4
    g, tables, phi = _case(nsteps)
    k_out = [k for k, io in enumerate(g.iolets) if io.kind == G.PRESSURE][0]
    m = MODELS[model]
    weights = None if objective == "wss" else np.array([0.3 if io.kind == G.VELOCITY else 1.0 for io in g.iolets])
    say(f"case: tortuous {g.n} sites, Windkessel {model} on iolet {k_out}, objective {objective}, "
        f"{nsteps} steps, {n_snap} checkpoints")
    P = oracle.Problem(g, tau, tables=tables, phi=phi)
    Jr, dAr, dphir = P.adjoint(P.init(), 0, nsteps, w0, w1, weights=weights, windkessel={k_out: m})
    sim = hlb.Simulation.create(g, tau, tables=tables, adjoint=True)
    hlb.hlb_set_porosity(sim.ctx, phi)
    hlb.hlb_set_windkessel(sim.ctx, k_out, m)
    if weights is not None:
        hlb.hlb_set_objective(sim.ctx, hlb.HLB_OBJ_IOLET_FLUX, weights)
    before = hlb.hlb_windkessel_state(sim.ctx, k_out)
    J, dA, dphi, fw = hlb.hlb_adjoint_run(sim.ctx, nsteps, w0, w1, n_snap)
    after = hlb.hlb_windkessel_state(sim.ctx, k_out)
    rows = ", ".join("%.2e" % rel(dA[k], dAr[k]) for k in range(len(g.iolets)))
    say(f"windkessel adjoint {model} {objective}: J {J:.10e} vs {Jr:.10e}; table rows rel {rel(dA, dAr):.2e} "
        f"({rows}); dphi rel {rel(dphi, dphir):.2e}; forward steps {fw}")
    assert abs(J - Jr) <= 1e-12 * abs(Jr)
    assert rel(dA, dAr) <= 1e-10
    assert rel(dA[k_out], dAr[k_out]) <= 1e-10
    assert rel(dphi, dphir) <= 1e-10
    assert np.allclose(before, after, rtol=0, atol=0)
    assert hlb.hlb_time(sim.ctx) == 0
    # the model matters: the same run with a constant outlet differs
    P0 = oracle.Problem(g, tau, tables=tables, phi=phi)
    J0 = P0.adjoint(P0.init(), 0, nsteps, w0, w1, weights=weights)[0]
    assert abs(J0 - Jr) > 1e-9 * abs(Jr)
    sim.close()
