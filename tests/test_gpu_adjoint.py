"""GPU adjoint (hlb_adjoint_run) against the oracle's reference adjoint and
central finite differences of the GPU forward objective.

Objective: J = sum over t in the window of the wall shear stress summed over
the sites with wall links; parameters: per-step inlet amplitudes (through 32
Fourier coefficients in the full case), per-step outlet ghost densities and
per-wall-site porosity.

The outlet density varies slightly around rho0 in the cases compared with
the oracle: at exactly rho0, a flow started from rest leaves sites whose
tangential traction is exactly zero, where the WSS magnitude has a kink; the
ghost-density derivative there depends on rounding (a 1e-14 change of the
outlet density moves it by ~10% in the oracle itself).
"""
import math
import sys
import time

import numpy as np
import pytest

import oracle
from paper_2202_11770_amd import geometry as G
from paper_2202_11770_amd import hlb

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


def _small_case(nsteps=60, seed=4):
    g = G.tortuous(radius=4.0, length=32, amplitude=4.0, period=32.0)
    rng = np.random.default_rng(seed)
    s = np.arange(nsteps)
    a = rng.uniform(-1, 1, 4) * 0.002 / np.arange(1, 5)
    b = rng.uniform(-1, 1, 4) * 0.002 / np.arange(1, 5)
    A = 0.01 + sum(a[k] * np.cos(2 * np.pi * (k + 1) * s / nsteps) + b[k] * np.sin(2 * np.pi * (k + 1) * s / nsteps)
                   for k in range(4))
    R = 1.0 + 0.001 * np.sin(2 * np.pi * s / nsteps)
    tables = [A if io.kind == G.VELOCITY else R.copy() for io in g.iolets]
    phi = np.zeros(g.n)
    ws = g.wall_sites()
    phi[ws] = np.random.default_rng(40).uniform(0, 1, ws.size)
    return g, tables, phi, ws


def _gpu_sim(g, tau, tables, phi):
    sim = hlb.Simulation.create(g, tau, tables=tables, adjoint=True)
    if phi is not None:
        hlb.hlb_set_porosity(sim.ctx, phi)
    return sim


class GpuObjective:
    """J by the GPU forward update: WSS summed on the device each window step."""

    def __init__(self, sim):
        import torch
        self.torch = torch
        self.sim = sim
        self.wss = torch.empty(sim.n, dtype=torch.float64, device="cuda")
        hlb.hlb_set_stream(sim.ctx, torch.cuda.current_stream().cuda_stream)

    def __call__(self, n, w0, w1, tables=None, phi=None):
        torch = self.torch
        ctx = self.sim.ctx
        if tables is not None:
            for k, t in enumerate(tables):
                hlb.hlb_set_iolet_table(ctx, k, t)
        if phi is not None:
            hlb.hlb_set_porosity(ctx, phi)
        hlb.hlb_init_equilibrium(ctx, None, None, 0)
        acc = torch.zeros((), dtype=torch.float64, device="cuda")
        first = max(w0, 0)
        if first > 0:
            hlb.hlb_step(ctx, min(first, n))
        for t in range(first + 1, min(w1, n) + 1):
            hlb.hlb_step(ctx, 1)
            hlb.hlb_macros_device(ctx, wss=self.wss)
            acc += self.wss.sum()
        if min(w1, n) < n:
            hlb.hlb_step(ctx, n - min(w1, n))
        return float(acc.item())


@pytest.mark.parametrize("porous", [True, False], ids=["porous", "no_porosity"])
def test_adjoint_matches_oracle_small(porous):
    """Without a porosity field the porosity derivative (at zero porosity)
    takes another kernel path: the collision part in k_adj_collide, the
    objective's part in k_adj_boundary."""
    nsteps, w0, w1, tau = 60, 30, 60, 0.8
    g, tables, phi, ws = _small_case(nsteps)
    if not porous:
        phi = None
    say(f"case: small tortuous {g.n} sites, porous {porous}")
    P = oracle.Problem(g, tau, tables=tables, phi=phi)
    Jr, dAr, dphir = P.adjoint(P.init(), 0, nsteps, w0, w1)
    sim = _gpu_sim(g, tau, tables, phi)
    J, dA, dphi, fw = hlb.hlb_adjoint_run(sim.ctx, nsteps, w0, w1, 4)
    say(f"small adjoint: J {J:.6e} vs {Jr:.6e}; table rows rel {rel(dA, dAr):.2e} "
        f"({', '.join('%.2e' % rel(dA[k], dAr[k]) for k in range(len(g.iolets)))}); "
        f"dphi rel {rel(dphi, dphir):.2e}; forward steps {fw}")
    assert abs(J - Jr) <= 1e-12 * abs(Jr)
    assert rel(dA, dAr) <= 1e-10
    assert rel(dphi, dphir) <= 1e-10
    assert hlb.hlb_time(sim.ctx) == 0
    sim.close()


@pytest.mark.parametrize("objective", ["wss", "flux"])
def test_device_outputs_and_setters_match_host(objective):
    """hlb_adjoint_run_device (device J, dJ/dA, dJ/dphi, asynchronous) and
    the device-array setters (table, porosity) give what the host forms
    give: the porosity gradient bit for bit, J and the table-value rows to
    the rounding of their atomic sums (whose order varies from run to run);
    a second call with another table and porosity, set from device arrays
    of the same length, overwrites the library's tables in place and still
    matches the host call."""
    import torch
    nsteps, w0, w1, tau = 60, 30, 60, 0.8
    g, tables, phi, ws = _small_case(nsteps)
    kind = hlb.HLB_OBJ_WSS if objective == "wss" else hlb.HLB_OBJ_IOLET_FLUX
    weights = None if objective == "wss" else np.linspace(0.5, 1.5, len(g.iolets))
    say(f"case: device vs host adjoint outputs, small tortuous {g.n} sites, objective {objective}")
    sim_h = _gpu_sim(g, tau, tables, phi)
    hlb.hlb_set_objective(sim_h.ctx, kind, weights)
    sim_d = _gpu_sim(g, tau, [np.ones(1) * (0.01 if io.kind == G.VELOCITY else 1.0) for io in g.iolets], None)
    hlb.hlb_set_objective(sim_d.ctx, kind, weights)
    hlb.hlb_set_stream(sim_d.ctx, torch.cuda.current_stream().cuda_stream)
    rng = np.random.default_rng(9)
    for trial in range(2):
        if trial == 1:
            tables = [t * (1.0 + 1e-3 * rng.uniform(-1, 1, t.size)) for t in tables]
            phi = phi * rng.uniform(0.5, 1.0, phi.size)
            for k, t in enumerate(tables):
                hlb.hlb_set_iolet_table(sim_h.ctx, k, t)
            hlb.hlb_set_porosity(sim_h.ctx, phi)
        for k, t in enumerate(tables):
            hlb.hlb_set_iolet_table_device(sim_d.ctx, k, torch.tensor(t, dtype=torch.float64, device="cuda"))
        hlb.hlb_set_porosity_device(sim_d.ctx, torch.tensor(phi, dtype=torch.float64, device="cuda"))
        J, dA, dphi, fw = hlb.hlb_adjoint_run(sim_h.ctx, nsteps, w0, w1, 4)
        Jd = torch.zeros(1, dtype=torch.float64, device="cuda")
        dAd = torch.zeros(len(g.iolets), nsteps, dtype=torch.float64, device="cuda")
        dphid = torch.zeros(g.n, dtype=torch.float64, device="cuda")
        fwd = hlb.hlb_adjoint_run_device(sim_d.ctx, nsteps, w0, w1, 4, Jd, dAd, dphid)
        torch.cuda.synchronize()
        say(f"trial {trial}: J host {J:.15e} device {float(Jd[0]):.15e}; forward steps {fw} / {fwd}")
        assert fwd == fw
        assert abs(float(Jd[0]) - J) <= 1e-14 * abs(J)
        assert np.abs(dAd.cpu().numpy() - dA).max() <= 1e-14 * np.abs(dA).max()
        assert np.array_equal(dphid.cpu().numpy(), dphi)
    # the checks reject out-of-range device values and change nothing
    bad = torch.tensor(phi, dtype=torch.float64, device="cuda")
    bad[ws[0]] = 1.5
    with pytest.raises(hlb.HLBError, match="porosity"):
        hlb.hlb_set_porosity_device(sim_d.ctx, bad)
    k_p = [k for k, io in enumerate(g.iolets) if io.kind == G.PRESSURE][0]
    badt = torch.tensor(tables[k_p], dtype=torch.float64, device="cuda")
    badt[3] = -1.0
    with pytest.raises(hlb.HLBError, match="ghost density"):
        hlb.hlb_set_iolet_table_device(sim_d.ctx, k_p, badt)
    badt[3] = float("nan")
    with pytest.raises(hlb.HLBError):
        hlb.hlb_set_iolet_table_device(sim_d.ctx, 0, badt)
    Jd2 = torch.zeros(1, dtype=torch.float64, device="cuda")
    hlb.hlb_adjoint_run_device(sim_d.ctx, nsteps, w0, w1, 4, Jd2)
    torch.cuda.synchronize()
    assert abs(float(Jd2[0]) - float(Jd[0])) <= 1e-14 * abs(float(Jd[0]))
    # hlb_stats: eq. (9) rate and algorithmic bandwidth over the timed steps
    hlb.hlb_set_timing(sim_h.ctx, True)
    sim_h.step(20)
    st = hlb.hlb_stats(sim_h.ctx)
    info = hlb.hlb_info(sim_h.ctx)
    assert st["steps"] == 20 and st["mlups"] > 0 and st["alg_gbs"] > 0
    assert abs(st["mlups"] - g.n / (st["step_ms"] * 1e3)) <= 1e-9 * st["mlups"]
    assert abs(st["alg_gbs"] - info["bytes_per_lup"] * g.n / (st["kernel_ms"] * 1e6)) <= 1e-9 * st["alg_gbs"]
    sim_h.close()
    sim_d.close()


def test_checkpoint_count_does_not_change_result():
    nsteps, w0, w1, tau = 60, 20, 50, 0.8
    g, tables, phi, ws = _small_case(nsteps)
    sim = _gpu_sim(g, tau, tables, phi)
    ref = hlb.hlb_adjoint_run(sim.ctx, nsteps, w0, w1, nsteps + 1)
    assert ref[3] == nsteps - 1  # enough slots: one forward sweep
    for ns in (1, 2, 3, 7):
        out = hlb.hlb_adjoint_run(sim.ctx, nsteps, w0, w1, ns)
        say(f"n_snap {ns}: forward steps {out[3]}")
        assert out[3] == hlb.hlb_revolve_forward_steps(nsteps, ns)  # the optimal count
        assert abs(out[0] - ref[0]) <= 1e-14 * abs(ref[0])
        assert rel(out[1], ref[1]) <= 1e-13 and rel(out[2], ref[2]) <= 1e-13
    # the state is left where it was, so a plain step still matches
    rho0, _, _ = sim.macros()
    assert np.abs(rho0 - 1.0).max() <= 1e-15
    sim.close()


def test_adjoint_vs_gpu_finite_differences():
    nsteps, w0, w1, tau = 60, 30, 60, 0.8
    g, tables, phi, ws = _small_case(nsteps)
    sim = _gpu_sim(g, tau, tables, phi)
    J, dA, dphi, _ = hlb.hlb_adjoint_run(sim.ctx, nsteps, w0, w1, 5)
    Jf = GpuObjective(sim)
    assert abs(Jf(nsteps, w0, w1) - J) <= 1e-12 * J
    k = [i for i, io in enumerate(g.iolets) if io.kind == G.VELOCITY][0]
    h = 1e-7
    steps = list(range(0, nsteps, 4))
    fd = []
    for s in steps:
        tp = [t.copy() for t in tables]
        tm = [t.copy() for t in tables]
        tp[k][s] += h
        tm[k][s] -= h
        fd.append((Jf(nsteps, w0, w1, tables=tp) - Jf(nsteps, w0, w1, tables=tm)) / (2 * h))
    Jf(nsteps, w0, w1, tables=tables)
    e_a = rel(dA[k, steps], fd)
    v = np.zeros(g.n)
    v[ws] = np.random.default_rng(9).uniform(-1, 1, ws.size)
    hp = 1e-6
    fdp = (Jf(nsteps, w0, w1, phi=phi + hp * v) - Jf(nsteps, w0, w1, phi=phi - hp * v)) / (2 * hp)
    e_p = abs(float(dphi @ v) - fdp) / abs(fdp)
    say(f"GPU FD: amplitude rel {e_a:.2e}, porosity direction rel {e_p:.2e}")
    assert e_a <= 1e-6 and e_p <= 1e-6
    sim.close()


def _c4(n_theta=32, seed=4):
    g = G.tortuous()  # radius 12, length 256
    rng = np.random.default_rng(seed)
    k = np.arange(1, n_theta // 2 + 1)
    theta = np.concatenate([rng.uniform(-1, 1, k.size) * 0.001 / k, rng.uniform(-1, 1, k.size) * 0.001 / k])
    phi = np.zeros(g.n)
    ws = g.wall_sites()
    phi[ws] = np.random.default_rng(40).uniform(0, 1, ws.size)
    return g, theta, phi, ws


def _inlet_np(theta, n, period):
    m = theta.size // 2
    s = np.arange(n)
    return 0.01 + sum(theta[j] * np.cos(2 * np.pi * (j + 1) * s / period) +
                      theta[m + j] * np.sin(2 * np.pi * (j + 1) * s / period) for j in range(m))


def test_c4_full_protocol_autograd_vs_fd():
    """Tortuous vessel (radius 12, length 256, ~1.25e5 sites), tau 0.8, 3000
    steps, J = time-integrated WSS over the last 500, 32 Fourier inlet
    coefficients and per-wall-site porosity, 30 snapshots; gradients through
    torch.autograd vs central FD (h = 1e-6) of the GPU forward objective."""
    import torch
    from paper_2202_11770_amd.autograd import WssObjective, fourier_inlet
    g, theta0, phi0, ws = _c4()
    n, w0, w1, tau, n_snap = 3000, 2500, 3000, 0.8, 30
    say(f"case: C4 tortuous {g.n} sites, {ws.size} wall sites, {n} steps, window ({w0},{w1}], {n_snap} snapshots")
    kinds = [io.kind for io in g.iolets]
    tables = [np.array([0.0]) if k == G.VELOCITY else np.array([1.0]) for k in kinds]
    sim = hlb.Simulation.create(g, tau, tables=tables, adjoint=True)
    # parameters on the GPU: the objective keeps them, J and the gradients there
    theta = torch.tensor(theta0, dtype=torch.float64, device="cuda", requires_grad=True)
    phi = torch.tensor(phi0, dtype=torch.float64, device="cuda", requires_grad=True)
    t = time.time()
    A = fourier_inlet(theta, n, period=float(n))[None, :]
    J = WssObjective.apply(A, phi, sim, n, w0, w1, n_snap)
    J.backward()
    t_adj = time.time() - t
    say(f"adjoint: J = {J.item():.8e} in {t_adj:.2f}s")
    assert J.is_cuda and theta.grad.is_cuda and phi.grad.is_cuda
    g_theta = theta.grad.cpu().numpy().copy()
    g_phi = phi.grad.cpu().numpy().copy()
    Jf = GpuObjective(sim)
    vel = kinds.index(G.VELOCITY)

    def J_of(th, ph):
        tabs = [t.copy() for t in tables]
        tabs[vel] = _inlet_np(th, n, float(n))
        return Jf(n, w0, w1, tables=tabs, phi=ph)

    J0 = J_of(theta0, phi0)
    assert abs(J0 - J.item()) <= 1e-12 * abs(J0)
    h = 1e-6
    t = time.time()
    fd = np.empty(theta0.size)
    for j in range(theta0.size):
        e = np.zeros(theta0.size)
        e[j] = h
        fd[j] = (J_of(theta0 + e, phi0) - J_of(theta0 - e, phi0)) / (2 * h)
    e_theta = rel(g_theta, fd)
    say(f"theta (32 components): rel err {e_theta:.2e}  ({time.time() - t:.1f}s for FD)")
    rng = np.random.default_rng(3)
    e_dir = []
    for _ in range(3):
        v = np.zeros(g.n)
        v[ws] = rng.uniform(-1, 1, ws.size)
        v /= np.abs(v).max()
        fdv = (J_of(theta0, phi0 + h * v) - J_of(theta0, phi0 - h * v)) / (2 * h)
        e_dir.append(abs(float(g_phi @ v) - fdv) / abs(fdv))
    say(f"porosity directions: rel errs {['%.2e' % x for x in e_dir]}")
    top = np.argsort(-np.abs(g_phi))[:16]
    fdt = []
    for x in top:
        v = np.zeros(g.n)
        v[x] = 1.0
        fdt.append((J_of(theta0, phi0 + h * v) - J_of(theta0, phi0 - h * v)) / (2 * h))
    e_top = rel(g_phi[top], fdt)
    say(f"16 largest porosity components: rel err {e_top:.2e}")
    assert e_theta <= 1e-6 and max(e_dir) <= 1e-6 and e_top <= 1e-6
    sim.close()


def test_c4_reduced_vs_oracle_adjoint():
    """The C4 geometry and parameters over 300 steps (window (250, 300]):
    GPU adjoint vs the oracle's reference adjoint, which keeps every state."""
    g, theta0, phi0, ws = _c4()
    n, w0, w1, tau = 300, 250, 300, 0.8
    A = _inlet_np(theta0, n, 3000.0)
    R = 1.0 + 0.001 * np.sin(2 * np.pi * np.arange(n) / n)
    tables = [A if io.kind == G.VELOCITY else R for io in g.iolets]
    P = oracle.Problem(g, tau, tables=tables, phi=phi0)
    t = time.time()
    Jr, dAr, dphir = P.adjoint(P.init(), 0, n, w0, w1)
    say(f"oracle adjoint {g.n} sites x {n} steps in {time.time() - t:.1f}s")
    sim = _gpu_sim(g, tau, tables, phi0)
    J, dA, dphi, fw = hlb.hlb_adjoint_run(sim.ctx, n, w0, w1, 10)
    say(f"C4 reduced: J rel {abs(J - Jr) / Jr:.2e}, dA rel {rel(dA, dAr):.2e}, dphi rel {rel(dphi, dphir):.2e}, "
        f"forward steps {fw}")
    assert abs(J - Jr) <= 1e-12 * Jr
    assert rel(dA, dAr) <= 1e-10 and rel(dphi, dphir) <= 1e-10
    sim.close()
