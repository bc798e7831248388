"""hlb_mass_balance_noalloc: the FP64 mass balance for callers that cannot
allocate (graph capture, serving loops), through the C ABI, against
hlb_mass_balance on the same state: bit for bit, two calls in a row, the
second on a smaller state, in every storage."""
import numpy as np
import pytest

from paper_2202_11770_amd import geometry as G
from paper_2202_11770_amd import hlb

pytestmark = pytest.mark.gpu


def _tables(g, period=200):
    s = np.arange(period)
    return [0.02 * 0.5 * (1 - np.cos(2 * np.pi * s / period)) if io.kind == G.VELOCITY else
            1.0 + 0.001 * np.sin(2 * np.pi * s / period) for io in g.iolets]


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_noalloc_mass_balance_matches_allocating_call(storage):
    import torch
    cases = [(G.tree(seed=3, generations=3, target_sites=30000), 0.6, 150),  # 30k sites
             (G.cylinder(), 0.8, 100)]                                      # then 13k sites
    for g, tau, steps in cases:
        print(f"case: no-alloc mass balance, {g.n} sites, {steps} steps, {storage}", flush=True)
        sim = hlb.Simulation.create(g, tau, storage=storage, tables=_tables(g))
        hlb.hlb_set_stream(sim.ctx, torch.cuda.current_stream().cuda_stream)
        sim.step(steps)
        out = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
        before = hlb.hlb_info(sim.ctx)["device_bytes"]
        hlb.hlb_mass_balance_noalloc(sim.ctx, out)
        torch.cuda.synchronize()
        assert hlb.hlb_info(sim.ctx)["device_bytes"] == before  # the context allocated nothing
        got = out.cpu().numpy()
        m, r = hlb.hlb_mass_balance(sim.ctx)
        print(f"no-alloc M {got[0]!r} R {got[1]!r}; allocating M {m!r} R {r!r}", flush=True)
        assert np.isfinite(got).all()
        assert got[0] == m and got[1] == r
        # the state moves on; the same output buffer is reused
        sim.step(7)
        hlb.hlb_mass_balance_noalloc(sim.ctx, out)
        torch.cuda.synchronize()
        m2, r2 = hlb.hlb_mass_balance(sim.ctx)
        assert out[0].item() == m2 and out[1].item() == r2
        sim.close()
