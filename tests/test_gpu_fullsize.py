"""Parity at the benchmark's full size and launch configuration.

The 2.0e7-site tree of the benchmark (seed 2, 8 generations, tau 0.6, one
Ladd inlet, 256 pressure outlets), default order and launch, every storage: a
few steps from the inlet-amplitude peak, every site compared against the
oracle; and the adjoint in the benchmark's configuration against central
differences of the GPU objective.

Every forward case starts from the same seeded non-uniform equilibrium on
both sides (rho = 1 +- 0.01, |u| <= 0.02 at every site), so that every site,
the far positions of the 64-bit address path included, holds populations
that no other site holds: a gather from a wrong site, or a wrong direction,
changes the result wherever it happens.
"""
import sys
import time

import numpy as np
import pytest

import oracle
from paper_2202_11770_amd import hlb
from _parity import check_bars, errors, fmt, random_field

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tree20m():
    sys.path.insert(0, ".")
    import bench
    t = time.time()
    g, tables = bench.tree_workload()
    print(f"tree {g.n} sites generated in {time.time() - t:.1f}s", flush=True)
    return g, tables


def test_tree_20m_parity(tree20m):
    """Every storage against one oracle run: FP64 to 1e-12; FP32 and FP16
    to bars about 3x above their measured errors."""
    g, tables = tree20m
    t0, steps, tau = 1000, 6, 0.6  # start at the inlet amplitude's peak
    rho0, u0 = random_field(g.n, 11)
    P = oracle.Problem(g, tau, tables=tables)
    f = P.init(rho0, u0)
    t = time.time()
    P.run(f, t0, steps)
    print(f"oracle {steps} steps in {time.time() - t:.1f}s", flush=True)
    ref = P.macros(f)
    m_ref = P.mass(f)
    del f
    for st in ("f64", "f32", "f16"):
        print(f"case: tree {g.n} sites, random start, t0 {t0}, {steps} steps, {st}, default launch", flush=True)
        sim = hlb.Simulation.create(g, tau, storage=st, tables=tables)
        hlb.hlb_init_equilibrium(sim.ctx, rho0, u0, t0)
        sim.step(steps)
        rho, u, wss = sim.macros()
        m, r = hlb.hlb_mass_balance(sim.ctx)
        sim.close()
        e = errors(rho, u, wss, *ref)
        print(f"tree20m {st}:", fmt(e), flush=True)
        if st == "f64":
            assert e["e_rho"] <= 1e-12 and e["e_u"] <= 1e-12 and e["e_wss"] <= 1e-10
            assert abs(m - m_ref) / m <= 1e-12
            assert abs(r) / m <= steps * 19 * 2.0 ** -53 / tau
        elif st == "f32":
            check_bars(e, dict(e_rho=5e-8, e_u=1e-6, e_wss=2e-6), "tree20m f32")
        else:
            check_bars(e, dict(e_rho=5e-5, e_u=1e-3, e_wss=2e-3), "tree20m f16")


def test_tree_20m_adjoint_vs_finite_differences(tree20m):
    """The adjoint in the benchmark's configuration (40 steps from rest, WSS
    summed over (20, 40], 10 checkpoints), checked at full size where the
    oracle's adjoint is out of reach: directional derivatives along a random
    perturbation of the per-step inlet amplitudes and of the wall porosity
    against central differences of the GPU objective."""
    g, tables = tree20m
    n, w0, w1, n_snap, tau = 40, 20, 40, 10, 0.6
    k_in = [k for k, io in enumerate(g.iolets) if io.kind == 0][0]
    rng = np.random.default_rng(7)
    walls = g.wall_sites()
    phi0 = np.zeros(g.n)
    phi0[walls] = 0.05
    v_phi = np.zeros(g.n)
    v_phi[walls] = rng.uniform(0, 1, walls.size)
    v_amp = rng.uniform(-1, 1, n)

    def run(amp_shift=None, phi=phi0, grads=False):
        tabs = [t.copy() for t in tables]
        if amp_shift is not None:
            tabs[k_in][:n] += amp_shift
        sim = hlb.Simulation.create(g, tau, tables=tabs, adjoint=True)
        hlb.hlb_set_porosity(sim.ctx, phi)
        J, dA, dphi, _ = hlb.hlb_adjoint_run(sim.ctx, n, w0, w1, n_snap, want_dA=grads, want_dphi=grads)
        sim.close()
        return J, dA, dphi

    print(f"case: tree {g.n} sites, adjoint {n} steps, window ({w0}, {w1}], {n_snap} checkpoints", flush=True)
    J, dA, dphi = run(grads=True)
    h = 1e-8
    fd = (run(amp_shift=h * v_amp)[0] - run(amp_shift=-h * v_amp)[0]) / (2 * h)
    ad = float(np.dot(dA[k_in], v_amp))
    e_amp = abs(fd - ad) / abs(fd)
    # J sums about 6e7 wall-site terms, whose rounding moves with any change
    # of the porosity: a step study on this case gives FD-vs-adjoint errors
    # of 1.6e-9 (h = 1e-4), 4.1e-8 (1e-5), 2.8e-6 (1e-6), 3.6e-5 (1e-7) --
    # rounding, growing as 1/h
    h = 1e-4
    fdp = (run(phi=phi0 + h * v_phi)[0] - run(phi=phi0 - h * v_phi)[0]) / (2 * h)
    adp = float(np.dot(dphi, v_phi))
    e_phi = abs(fdp - adp) / abs(fdp)
    print(f"J {J:.10e}; amplitudes: adjoint {ad:.10e} FD {fd:.10e} rel {e_amp:.1e}; "
          f"porosity: adjoint {adp:.10e} FD {fdp:.10e} rel {e_phi:.1e}", flush=True)
    assert e_amp <= 1e-6 and e_phi <= 1e-6


def test_tree_30m_fp64_wide_addressing_parity():
    """Above 4 GiB per population buffer the step kernel forms 64-bit
    addresses instead of 32-bit offsets from a scalar base.  A 3.0e7-site
    tree in FP64 (4.6 GB per buffer) takes that path; every site is
    compared against the oracle after a few steps from the inlet peak, from
    a random start."""
    sys.path.insert(0, ".")
    import bench
    t = time.time()
    g, tables = bench.tree_workload(target=30_000_000)
    print(f"tree {g.n} sites generated in {time.time() - t:.1f}s", flush=True)
    t0, steps, tau = 1000, 4, 0.6
    sim = hlb.Simulation.create(g, tau, tables=tables)
    info = hlb.hlb_info(sim.ctx)
    assert 19 * info["n_padded"] * 8 > 2 ** 32, "the case must exceed 4 GiB per buffer"
    print(f"case: tree {g.n} sites ({19 * info['n_padded'] * 8 / 1e9:.2f} GB per buffer), t0 {t0}, {steps} steps, f64",
          flush=True)
    rho0, u0 = random_field(g.n, 12)
    hlb.hlb_init_equilibrium(sim.ctx, rho0, u0, t0)
    sim.step(steps)
    rho, u, wss = sim.macros()
    sim.close()
    P = oracle.Problem(g, tau, tables=tables)
    f = P.init(rho0, u0)
    del rho0, u0
    P.run(f, t0, steps)
    e = errors(rho, u, wss, *P.macros(f))
    print("tree30m f64:", fmt(e), flush=True)
    assert e["e_rho"] <= 1e-12 and e["e_u"] <= 1e-12 and e["e_wss"] <= 1e-10


def test_tree_120m_fp16_wide_addressing_parity():
    """The same for FP16 storage, which crosses 4 GiB per buffer only above
    1.13e8 sites: a 1.2e8-site tree, against the oracle at every site, to
    the FP16 storage bound."""
    sys.path.insert(0, ".")
    import bench
    t = time.time()
    g, tables = bench.tree_workload(target=120_000_000)
    print(f"tree {g.n} sites generated in {time.time() - t:.1f}s", flush=True)
    t0, steps, tau = 1000, 4, 0.6
    sim = hlb.Simulation.create(g, tau, storage="f16", tables=tables)
    info = hlb.hlb_info(sim.ctx)
    assert 19 * info["n_padded"] * 2 > 2 ** 32, "the case must exceed 4 GiB per buffer"
    print(f"case: tree {g.n} sites ({19 * info['n_padded'] * 2 / 1e9:.2f} GB per buffer), t0 {t0}, {steps} steps, f16",
          flush=True)
    rho0, u0 = random_field(g.n, 13)
    hlb.hlb_init_equilibrium(sim.ctx, rho0, u0, t0)
    sim.step(steps)
    rho, u, wss = sim.macros()
    sim.close()
    P = oracle.Problem(g, tau, tables=tables)
    f = P.init(rho0, u0)
    del rho0, u0
    t = time.time()
    P.run(f, t0, steps)
    print(f"oracle {steps} steps in {time.time() - t:.1f}s", flush=True)
    e = errors(rho, u, wss, *P.macros(f))
    print("tree120m f16:", fmt(e), flush=True)
    check_bars(e, dict(e_rho=5e-5, e_u=1e-3, e_wss=2e-3), "tree120m f16")


def test_tree_200m_fp64_parity():
    """The 2.0e8-site tree of the large workload (30 GB per FP64 buffer),
    default launch: every site against the oracle after a few steps from the
    inlet peak (the oracle needs about 80 GB of host memory here)."""
    sys.path.insert(0, ".")
    import bench
    t = time.time()
    g, tables = bench.workload("tree200m")
    print(f"tree {g.n} sites generated in {time.time() - t:.1f}s", flush=True)
    t0, steps, tau = 1000, 3, 0.6
    print(f"case: tree {g.n} sites, t0 {t0}, {steps} steps, f64", flush=True)
    sim = hlb.Simulation.create(g, tau, tables=tables)
    rho0, u0 = random_field(g.n, 14)
    hlb.hlb_init_equilibrium(sim.ctx, rho0, u0, t0)
    sim.step(steps)
    rho, u, wss = sim.macros()
    sim.close()
    P = oracle.Problem(g, tau, tables=tables)
    f = P.init(rho0, u0)
    del rho0, u0
    t = time.time()
    P.run(f, t0, steps)
    print(f"oracle {steps} steps in {time.time() - t:.1f}s", flush=True)
    e = errors(rho, u, wss, *P.macros(f))
    print("tree200m f64:", fmt(e), flush=True)
    assert e["e_rho"] <= 1e-12 and e["e_u"] <= 1e-12 and e["e_wss"] <= 1e-10
