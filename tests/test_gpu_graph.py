"""Replayed HIP graphs in hlb_step (hlb_options.graph_steps) against plain
launches.

A graph holds a fixed number of steps and reads the starting time from
device memory, so one graph serves every starting time.  Each case runs the
same sequence of hlb_step calls -- whole graphs, remainders, calls shorter
than a graph -- with eager work between them (macros, table changes,
porosity, a state reset), and compares every intermediate result with the
plain-launch run bit for bit.
"""
import numpy as np
import pytest

from paper_2202_11770_amd import geometry as G
from paper_2202_11770_amd import hlb

pytestmark = pytest.mark.gpu

CALLS = [100, 64, 7, 200, 2, 129]


def _case():
    g = G.cylinder()
    # table lengths that do not divide the graph length: the replays must
    # read the right entry at every starting time
    tables = [0.01 * (1 + 0.5 * np.sin(2 * np.pi * np.arange(37) / 37)) if io.kind == G.VELOCITY else
              1.0 + 0.001 * np.cos(2 * np.pi * np.arange(53) / 53) for io in g.iolets]
    return g, tables


def _run(graph_steps, storage="f64", scheme="pull", windkessel=False, porous=False):
    g, tables = _case()
    sim = hlb.Simulation.create(g, 0.8, storage=storage, tables=tables, scheme=scheme, graph_steps=graph_steps)
    info = hlb.hlb_info(sim.ctx)
    out = []
    if windkessel:
        k = [k for k, io in enumerate(g.iolets) if io.kind == G.PRESSURE][0]
        hlb.hlb_set_windkessel(sim.ctx, k, (1.0, 0.002, 500.0, 0.004, 0.0))
    for j, n in enumerate(CALLS):
        sim.step(n)
        out.append(sim.macros())
        out.append(hlb.hlb_get_state(sim.ctx))
        if j == 1:
            # new inlet table (same length) between calls
            k_in = [k for k, io in enumerate(g.iolets) if io.kind == G.VELOCITY][0]
            hlb.hlb_set_iolet_table(sim.ctx, k_in, 0.015 * np.ones(37))
        if j == 2 and porous:
            phi = np.zeros(g.n)
            ws = g.wall_sites()
            phi[ws] = np.random.default_rng(2).uniform(0, 0.2, ws.size)
            hlb.hlb_set_porosity(sim.ctx, phi)
        if j == 3:
            # state reset to the state of an odd time: the next call starts
            # from the other buffer
            f = hlb.hlb_get_state(sim.ctx)
            hlb.hlb_set_state(sim.ctx, f, 371)
    m, r = hlb.hlb_mass_balance(sim.ctx)
    sim.close()
    return info, out, (m, r)


@pytest.mark.parametrize("graph_steps", [2, 64])
@pytest.mark.parametrize("variant", ["f64", "f32", "f16", "push", "windkessel", "porous"])
def test_graph_replays_match_plain_launches(variant, graph_steps):
    kw = dict(storage=variant if variant in ("f64", "f32", "f16") else "f64",
              scheme="push" if variant == "push" else "pull", windkessel=variant == "windkessel",
              porous=variant == "porous")
    print(f"case: cylinder {variant}, {graph_steps} steps per graph, calls {CALLS}", flush=True)
    info, a, (ma, ra) = _run(graph_steps, **kw)
    assert info["graph_steps"] == graph_steps
    info0, b, (mb, rb) = _run(0, **kw)
    assert info0["graph_steps"] == 0
    worst = 0.0
    for k, (x, y) in enumerate(zip(a, b)):
        xs = x if isinstance(x, tuple) else (x,)
        ys = y if isinstance(y, tuple) else (y,)
        for u, v in zip(xs, ys):
            if variant == "windkessel":
                # the outlet's outflow is summed with atomics in no fixed
                # order, so its ghost density -- and the flow -- vary in the
                # last bits between any two runs
                d = float(np.abs(u - v).max() / max(np.abs(v).max(), 1e-300))
                worst = max(worst, d)
                assert d <= 1e-12, f"result {k} differs by {d:.2e}"
            else:
                assert np.array_equal(u, v), f"result {k} differs"
    print(f"largest relative difference {worst:.2e}")
    # the mass is a fixed-order reduction of the state; the balance residual
    # also holds the boundary flux, which the step kernel sums with atomics in
    # no fixed order (plain launches vary the same way from run to run)
    assert ma == mb
    assert abs(ra - rb) <= 1e-13 * ma


def test_default_graph_steps_and_timing():
    g, tables = _case()
    assert hlb.hlb_info(hlb.Simulation.create(g, 0.8, tables=tables).ctx)["graph_steps"] == 0
    sim = hlb.Simulation.create(g, 0.8, tables=tables, graph_steps=64)
    assert hlb.hlb_info(sim.ctx)["graph_steps"] == 64
    # with timing on, every step is a plain launch with its own events
    hlb.hlb_set_timing(sim.ctx, True)
    sim.step(130)
    st = hlb.hlb_stats(sim.ctx)
    assert st["steps"] == 130
    hlb.hlb_set_timing(sim.ctx, False)
    sim.close()
