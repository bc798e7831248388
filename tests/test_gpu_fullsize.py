"""Parity at the benchmark's full size and launch configuration.

The 2.0e7-site tree of the benchmark (seed 2, 8 generations, tau 0.6, one
Ladd inlet, 256 pressure outlets), default order and launch, FP64: a few steps
from the inlet-amplitude peak, every site compared against the oracle.
"""
import sys
import time

import numpy as np
import pytest

import oracle
from paper_2202_11770_amd import hlb
from _parity import errors, fmt

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tree20m():
    sys.path.insert(0, ".")
    import bench
    t = time.time()
    g, tables = bench.tree_workload()
    print(f"tree {g.n} sites generated in {time.time() - t:.1f}s", flush=True)
    return g, tables


def test_tree_20m_fp64_parity(tree20m):
    g, tables = tree20m
    t0, steps, tau = 1000, 6, 0.6  # start at the inlet amplitude's peak
    print(f"case: tree {g.n} sites, t0 {t0}, {steps} steps, f64, default launch", flush=True)
    sim = hlb.Simulation.create(g, tau, tables=tables)
    hlb.hlb_init_equilibrium(sim.ctx, None, None, t0)
    sim.step(steps)
    rho, u, wss = sim.macros()
    m, r = hlb.hlb_mass_balance(sim.ctx)
    sim.close()
    P = oracle.Problem(g, tau, tables=tables)
    f = P.init()
    t = time.time()
    P.run(f, t0, steps)
    print(f"oracle {steps} steps in {time.time() - t:.1f}s", flush=True)
    e = errors(rho, u, wss, *P.macros(f))
    print("tree20m f64:", fmt(e), flush=True)
    assert e["e_rho"] <= 1e-12 and e["e_u"] <= 1e-12 and e["e_wss"] <= 1e-10
    assert abs(m - P.mass(f)) / m <= 1e-12
    assert abs(r) / m <= steps * 19 * 2.0 ** -53 / tau
