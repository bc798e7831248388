"""Error table on the error subtree of the 2.0e8-site tree.

The 2.0e8-site tree (seed 2, 8 generations) is never voxelised here: the
subtree rooted at the first child of the generation whose subtree is closest
to 2e6 sites is cut from the segment list and voxelised at the same lattice
spacing.  Its root gets its own Ladd inlet with the benchmark's amplitude
A(s); its leaves are rho = 1 pressure outlets; tau 0.6; 1000 steps from rest.
All three storages are compared with the FP64 oracle on every site.
"""
import sys
import time

import numpy as np
import pytest

import oracle
from paper_2202_11770_amd import geometry as G
from paper_2202_11770_amd import hlb
from _parity import check_bars, errors, fmt

pytestmark = pytest.mark.gpu

TAU, STEPS = 0.6, 1000


@pytest.fixture(scope="module")
def subtree_case():
    sys.path.insert(0, ".")
    import bench
    t = time.time()
    seg = G.tree_segments(2, 8, scale=bench.TREE_SCALE_200M, origin=(0.5, 0.5, -0.5))
    g = G.subtree(segments=seg, scale=bench.TREE_SCALE_200M, target_sites=2_000_000)
    tables = [bench.inlet_table() if io.kind == G.VELOCITY else np.array([1.0]) for io in g.iolets]
    print(f"subtree: generation {g.meta['generation']}, {g.n} sites, {len(g.iolets)} iolets, "
          f"built in {time.time() - t:.1f}s", flush=True)
    P = oracle.Problem(g, TAU, tables=tables)
    f = P.init()
    t = time.time()
    P.run(f, 0, STEPS)
    print(f"oracle {STEPS} steps in {time.time() - t:.1f}s", flush=True)
    return g, tables, P.macros(f), P.mass(f)


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_subtree_error_table(subtree_case, storage):
    g, tables, ref, mass_ref = subtree_case
    print(f"case: subtree {g.n} sites, {STEPS} steps, {storage}", flush=True)
    sim = hlb.Simulation.create(g, TAU, storage=storage, tables=tables)
    sim.step(STEPS)
    rho, u, wss = sim.macros()
    m, r = hlb.hlb_mass_balance(sim.ctx)
    sim.close()
    e = errors(rho, u, wss, *ref)
    print(f"subtree {storage}: {fmt(e)} mass_rel={(m - mass_ref) / mass_ref:.2e} "
          f"residual_rel={r / m:.2e}", flush=True)
    if storage == "f64":
        assert e["e_rho"] <= 1e-12 and e["e_u"] <= 1e-12 and e["e_wss"] <= 1e-10
        assert abs(m - mass_ref) / mass_ref <= 1e-12
    elif storage == "f32":
        check_bars(e, dict(e_rho=5e-7, e_u=2e-5, e_wss=3e-5), "subtree f32")
        assert e["e_rho"] <= 1e-5 and e["e_u"] <= 1e-5 and e["e_wss"] <= 1e-5  # the FP32 target
    else:
        check_bars(e, dict(e_rho=5e-5, e_u=2e-3, e_wss=1e-2), "subtree f16")
