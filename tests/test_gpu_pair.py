"""Two bulk+wall sites per GPU thread (hlb_options.sites_per_thread = 2)
against one site per thread.

Each site's update reads the same values and does the same arithmetic in
either form, so the two must agree bit for bit, in every storage, with and
without porous walls.  The cases have an odd and an even number of
256-position blocks in the bulk+wall group, so the last block pair is both
partial and full.
"""
import numpy as np
import pytest

from paper_2202_11770_amd import geometry as G
from paper_2202_11770_amd import hlb

pytestmark = pytest.mark.gpu


def _tree():
    g = G.tree(seed=3, generations=3, target_sites=30000)
    s = np.arange(200)
    tables = [0.02 * 0.5 * (1 - np.cos(2 * np.pi * s / 200)) if io.kind == G.VELOCITY else
              1.0 + 0.001 * np.sin(2 * np.pi * s / 200) for io in g.iolets]
    return g, tables


def _run(g, tables, storage, spt, steps, phi=None):
    sim = hlb.Simulation.create(g, 0.6, storage=storage, tables=tables, sites_per_thread=spt)
    if phi is not None:
        hlb.hlb_set_porosity(sim.ctx, phi)
    sim.step(steps)
    out = sim.macros()
    f = hlb.hlb_get_state(sim.ctx)
    m, _ = hlb.hlb_mass_balance(sim.ctx)
    sim.close()
    return out, f, m


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
@pytest.mark.parametrize("case", ["tree", "cylinder", "tree_porous"])
def test_two_sites_per_thread_bitwise(case, storage):
    if case == "cylinder":
        g, tables, phi = G.cylinder(), None, None
    else:
        g, tables = _tree()
        phi = None
        if case == "tree_porous":
            phi = np.zeros(g.n)
            ws = g.wall_sites()
            phi[ws] = np.random.default_rng(1).uniform(0, 0.3, ws.size)
    probe = hlb.Simulation.create(g, 0.6, storage=storage, tables=tables)
    n0 = hlb.hlb_info(probe.ctx)["group_sites"][0]
    probe.close()
    print(f"case: {case} {g.n} sites ({(n0 + 255) // 256} bulk blocks), {storage}", flush=True)
    a, fa, ma = _run(g, tables, storage, 1, 300, phi)
    b, fb, mb = _run(g, tables, storage, 2, 300, phi)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    assert np.array_equal(fa, fb)
    assert ma == mb
