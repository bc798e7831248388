"""Pins of the oracle's Windkessel outlets (Problem.run_windkessel; no GPU).

The model (not in the paper): rho_k(s+1) = rho_ref + R1 Q_k(s) + X(s+1),
X(s+1) = X(s) + (Q_k(s) - X(s)/R2)/C, or R2 Q_k(s) if C = 0, Q_k(s) the
outflow of the update s -> s+1 (orc_iolet_flux).  Pins:
  * R1 = R2 = C = 0 is a constant-density outlet: identical to the plain run;
  * steady state on the pipe: the outlet's outflow equals the Ladd inflow
    (mass conservation), X = R2 Q, rho = rho_ref + (R1 + R2) Q;
  * a pure capacitor (R1 = R2 = 0) integrates the outflow: C (X(T) - X0)
    is the summed outflow.
"""
import numpy as np

import oracle
from paper_2202_11770_amd import geometry as G


def _pipe():
    g = G.cylinder()
    k_out = [k for k, io in enumerate(g.iolets) if io.kind == G.PRESSURE][0]
    k_in = [k for k, io in enumerate(g.iolets) if io.kind == G.VELOCITY][0]
    return g, k_in, k_out


def test_zero_model_is_constant_outlet():
    g, _, k = _pipe()
    P = oracle.Problem(g, 0.8)
    f = P.init()
    P.run(f, 0, 200)
    P2 = oracle.Problem(g, 0.8)
    f2 = P2.init()
    st = P2.run_windkessel(f2, 0, 200, {k: (1.0, 0.0, 0.0, 0.0, 0.0)})
    assert np.array_equal(f, f2)
    assert st[k][0] == 1.0


def test_rcr_steady_state_on_pipe():
    g, k_in, k = _pipe()
    rho_ref, R1, C, R2 = 1.0, 0.001, 2000.0, 0.002
    P = oracle.Problem(g, 0.8)
    f = P.init()
    # the start-up transient decays on the viscous time R^2/nu = 640 steps
    st = P.run_windkessel(f, 0, 5000, {k: (rho_ref, R1, C, R2, 0.0)})
    rho_next, X, Q = st[k]
    Q_in = -P.iolet_flux(f, 5000)[k_in]
    print(f"outflow {Q:.6f} inflow {Q_in:.6f} X {X:.6e} R2 Q {R2 * Q:.6e} rho {rho_next:.8f}")
    assert abs(Q - Q_in) <= 2e-4 * Q_in
    assert abs(X - R2 * Q) <= 2e-4 * R2 * Q
    assert abs(rho_next - (rho_ref + (R1 + R2) * Q)) <= 1e-6


def test_capacitor_integrates_outflow():
    g, _, k = _pipe()
    C, X0 = 500.0, 0.001
    P = oracle.Problem(g, 0.8)
    f = P.init()
    # outflows step by step, from the same routine run one step at a time
    Qs = []
    for s in range(100):
        st = P.run_windkessel(f, s, 1, {k: (1.0, 0.0, C, 0.0, X0 + sum(Qs) / C)})
        Qs.append(st[k][2])
    P2 = oracle.Problem(g, 0.8)
    f2 = P2.init()
    rho_next, X, _ = P2.run_windkessel(f2, 0, 100, {k: (1.0, 0.0, C, 0.0, X0)})[k]
    assert abs(C * (X - X0) - sum(Qs)) <= 1e-12 * abs(sum(Qs))
    assert abs(rho_next - (1.0 + X)) <= 1e-15
